// k_xpass.hip -- transforms along x (steps 1 and 9 of the solve sequence in
// FluTAS Section 3.3.1), one workgroup per block of NB grid rows.
//
// Forward: a row of nx reals x[i] is read as M = nx/2 complex values
// z[n] = x[2n] + i x[2n+1]; an M-point FFT gives Z; the half spectrum of the
// real row follows from
//     X[m] = (Z[m] + conj Z[M-m])/2 - i w^m (Z[m] - conj Z[M-m])/2,
//     w = exp(-2 pi i/nx),  m = 1..M-1,
// and X[0] = Re Z[0] + Im Z[0], X[M] = Re Z[0] - Im Z[0] (both real), which
// are packed as S[0] = X[0] + i X[M].
// Optionally the input is the FP64 residual r = (f - mu) - L p of the
// iterative refinement, evaluated from f and p row by row into the LDS tile
// (its L2 norm and that of f - mu accumulate in FP64 per workgroup), so r
// never touches HBM.
//
// Inverse: Z'[m] = (X[m] + conj X[M-m]) + i w^-m (X[m] - conj X[M-m]) with
// Z'[0] = (X[0] + X[M]) + i (X[0] - X[M]); an inverse M-point FFT of Z'
// returns nx (x[2n] + i x[2n+1]) (unnormalised, like the forward pass), which
// is stored to p or added to it in FP64.
//
// Walls along x (the XW kernel variants): the rows are expanded in the
// cosine or sine modes of the wall condition through the same half spectrum
// of the reordered row (see wall_emit / wall_load below).  The projection
// step's forward pass takes the divergence of the face velocities as input.
//
// Compiled once per precision with PK_REAL = float or double.
#include <type_traits>

#include "fft_core.hpp"
#include "lengths.hpp"
#include "stencil.hpp"

#ifndef PK_REAL
#error "PK_REAL must be defined"
#endif

namespace pk {
namespace PK_NS {

using R = PK_REAL;

template <int M> struct XCfg {
    static constexpr int ELEMS = sizeof(R) == 4 ? 4096 : 2048;
    static constexpr int NB0 = ELEMS / M;
    static constexpr int NB = NB0 < 1 ? 1 : (NB0 > 64 ? 64 : NB0);
    static constexpr int NT = pick_nt(NB * M, sizeof(R) == 4 ? 16 : 8);
    static constexpr int PAD = 0;
};

// The split of the M-point spectrum (forward) and its merge (inverse) couple
// the values at m and M - m.  In the last Stockham pass (forward) and the
// first one (inverse) the butterfly j handles indices j + r NJ, r < RAD,
// NJ = M/RAD, and the partner of j + r NJ is (NJ - j) + (RAD-1-r) NJ for
// j > 0, while butterflies 0 and NJ/2 are their own partners (r <-> RAD-r and
// r <-> RAD-1-r).  A thread therefore takes the butterfly pair (p, NJ - p)
// for p in [1, NJ/2), or (0, NJ/2) for p = 0, and both values of every
// coupled pair meet in its registers: no extra LDS round trip in the forward
// pass, and every spectrum element is read once in the inverse pass.
template <int NJ>
__device__ __forceinline__ void pair_of(int p, int &j1, int &j2)
{
    j1 = p;
    j2 = (p == 0) ? NJ / 2 : NJ - p;
}

// forward split of one coupled pair: zm = Z[m], zc = Z[M-m], w = exp(-2 pi i m/nx)
//   X[m] = A + w B,  X[M-m] = conj(A - w B),
//   A = (zm + conj zc)/2,  B = -i (zm - conj zc)/2
template <typename T>
__device__ __forceinline__ void split_pair(Cx<T> zm, Cx<T> zc, Cx<T> w, Cx<T> &xm, Cx<T> &xc)
{
    const Cx<T> A = cscale(cadd(zm, cconj(zc)), T(0.5));
    const Cx<T> B = cscale(cmul_mi(csub(zm, cconj(zc))), T(0.5));
    const Cx<T> wB = cmul(w, B);
    xm = cadd(A, wB);
    xc = cconj(csub(A, wB));
}

// inverse merge of one coupled pair: xm = X[m], xc = X[M-m], w = exp(-2 pi i m/nx)
//   Z'[m] = A + T,  Z'[M-m] = conj(A - T),
//   A = xm + conj xc,  T = i conj(w) (xm - conj xc);
// returned conjugated (the inverse runs as conj(FFT(conj))).
template <typename T>
__device__ __forceinline__ void merge_pair(Cx<T> xm, Cx<T> xc, Cx<T> w, Cx<T> &zm, Cx<T> &zc)
{
    const Cx<T> A = cadd(xm, cconj(xc));
    const Cx<T> Tt = cmul_pi(cmul(cconj(w), csub(xm, cconj(xc))));
    zm = cconj(cadd(A, Tt));
    zc = csub(A, Tt);
}

// Walls along x (cosine basis for Neumann, sine basis for Dirichlet): a real
// row x of nx cells is read reordered, v[j] = x[r(j)] with r(j) = 2j (2j < nx)
// or 2nx-1-2j (and (-1)^r(j) x[r(j)] for sines), so the half spectrum X of v
// gives the coefficients (Makhoul's method)
//     C[k] = Re(w_k X[k]),  C[nx-k] = Re(w_{nx-k} conj X[k]),  w_k = exp(-i pi k/(2nx)),
// each X[k] yielding two; for sines coefficient k sits at nx-1-k.  They are
// stored in the real view of the row (coefficient k at real offset k), so a
// spectrum column m holds the real x-modes 2m and 2m+1 as C[2m] + i C[2m+1].
// The inverse reads W[k] = conj(w_k) (C[k] - i C[nx-k]) (C[nx] = 0; W is
// Hermitian, so the C2R merge applies), with W[0] + i W[M] = C[0] + i sqrt2
// C[M] in the packed column, and stores v[j] back to x[r(j)].
__device__ __forceinline__ int wall_index(int j, int nx) { return 2 * j < nx ? 2 * j : 2 * nx - 1 - 2 * j; }

template <typename T>
__device__ __forceinline__ void wall_emit(PK_GLOBAL T *row, int nx, int m, Cx<T> X,
                                          const Cx<T> *w4, bool sine)
{
    const Cx<T> wa = w4[m];
    row[sine ? nx - 1 - m : m] = wa.re * X.re - wa.im * X.im;  // Re(w_m X)
    // w_{nx-m} = -i conj(w_m), so Re(w_{nx-m} conj X) = -Im(w_m X): one
    // table entry serves both coefficients
    if (2 * m != nx) row[sine ? m - 1 : nx - m] = -(wa.re * X.im + wa.im * X.re);
}

// coefficient k of a wall row (real view), reversed for sines; C[nx] = 0
template <typename T>
__device__ __forceinline__ T wall_coef(const PK_GLOBAL T *row, int nx, int k, bool sine)
{
    if (k >= nx) return T(0);
    return row[sine ? nx - 1 - k : k];
}

// X[m] for the inverse pass from the coefficients of a wall row
template <typename T>
__device__ __forceinline__ Cx<T> wall_load(const PK_GLOBAL T *row, int nx, int m,
                                           const PK_GLOBAL Cx<T> *w4, bool sine)
{
    if (m == 0) return {wall_coef(row, nx, 0, sine), T(1.4142135623730951) * wall_coef(row, nx, nx / 2, sine)};
    const T a = wall_coef(row, nx, m, sine), b = wall_coef(row, nx, nx - m, sine);
    const Cx<T> w = w4[m];
    return {w.re * a - w.im * b, -(w.re * b + w.im * a)};
}

// Forward transform of the NB lines of M points held by a workgroup: pass 0
// reads through gload (from global memory, or from the tile itself when
// GL_LDS), and the last pass writes the half spectra of the real rows through
// out(b) (row pointer into S, null to skip the row).  LDS tile `tile` and the
// nx-entry twiddle table `tw` are the caller's; no trailing barrier.
// P0 = 1: the tile already holds the output of pass 0 (Pass0Regs), the
// transform continues from pass 1 (needs at least two passes).
template <int M, int NB, int NT, bool GL_LDS, int P0 = 0, bool XW = false, class GL, class OUT>
__device__ __forceinline__ void x_forward(const Cx<R> *tw, GL &gload, LdsTile<R, M, NB, false, 0> tile,
                                          OUT &out, bool sine = false, const Cx<R> *w4 = nullptr)
{
    auto lstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
    constexpr RPlan pl = make_rplan(M);
    static_assert(P0 == 0 || pl.count >= 2, "");
    if constexpr (pl.count >= 2) {
        // all passes but the last, then the last pass with the split fused
        if constexpr (pl.count - 1 > P0) {
            fft_passes<R, M, NB, NT, false, 0, GL_LDS, P0, pl.count - 1, 0>(tw, 2, gload, lstore,
                                                                            tile);
            __syncthreads();
        }
        constexpr int RAD = pl.r[pl.count - 1];
        constexpr int NJ = M / RAD;
        static_assert(NJ == rplan_ns(pl, pl.count - 1) && NJ % 2 == 0, "pairing needs even NJ");
        constexpr int U = NJ / 2, NU = NB * U;
        constexpr int PER = (NU + NT - 1) / NT;
        // walls: the basis (cosines or sines) is a compile-time constant of
        // each copy of the last pass, so that every coefficient store has a
        // fixed offset from its row pointer (a per-store select of the index
        // took 40 more registers)
        auto last_pass = [&](auto sine_c) {
            constexpr bool sine = decltype(sine_c)::value;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u / U, pp = u % U;
                int j1, j2;
                pair_of<NJ>(pp, j1, j2);
                Cx<R> v1[RAD], v2[RAD];
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    v1[r] = tile.at(b, j1 + r * NJ);
                    v2[r] = tile.at(b, j2 + r * NJ);
                }
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    v1[r] = cmul(v1[r], tw[2 * r * j1]);
                    v2[r] = cmul(v2[r], tw[2 * r * j2]);
                }
                Bfly<R, RAD>::run(v1);
                Bfly<R, RAD>::run(v2);
                PK_GLOBAL Cx<R> *Sr = out(b);
                if (!Sr) continue;
                PK_GLOBAL R *Sreal = (PK_GLOBAL R *)Sr;
                auto emit = [&](int m, Cx<R> zm, Cx<R> zc) {
                    Cx<R> xm, xc;
                    split_pair(zm, zc, tw[m], xm, xc);
                    if constexpr (XW) {
                        wall_emit(Sreal, 2 * M, m, xm, w4, sine);
                        if (2 * m != M) wall_emit(Sreal, 2 * M, M - m, xc, w4, sine);
                    } else {
                        put(Sr + m, xm);
                        if (2 * m != M) put(Sr + (M - m), xc);
                    }
                };
                if (pp == 0) {
                    // butterfly 0: m = r NJ; m = 0 packs X(0) + i X(M)
                    const R X0 = v1[0].re + v1[0].im, XM = v1[0].re - v1[0].im;
                    if constexpr (XW) {
                        Sreal[sine ? 2 * M - 1 : 0] = X0;
                        Sreal[sine ? M - 1 : M] = XM * w4[M].re;
                    } else {
                        put(Sr, Cx<R>{X0, XM});
                    }
#pragma unroll
                    for (int r = 1; r < RAD; ++r)
                        if (r <= RAD - r) emit(r * NJ, v1[r], v1[RAD - r]);
                    // butterfly NJ/2: m = NJ/2 + r NJ, partner r <-> RAD-1-r
#pragma unroll
                    for (int r = 0; r < RAD; ++r)
                        if (r <= RAD - 1 - r) emit(NJ / 2 + r * NJ, v2[r], v2[RAD - 1 - r]);
                } else {
#pragma unroll
                    for (int r = 0; r < RAD; ++r) emit(j1 + r * NJ, v1[r], v2[RAD - 1 - r]);
                }
            }
        };
        if constexpr (XW) {
            if (sine)
                last_pass(std::true_type{});
            else
                last_pass(std::false_type{});
        } else {
            last_pass(std::false_type{});
        }
    } else {
        fft_tile<R, M, NB, NT, false, 0, GL_LDS>(tw, 2, gload, lstore, tile);
        __syncthreads();
        // split the M-point spectrum into the half spectrum of the real rows
        for (int u = threadIdx.x; u < NB * M; u += NT) {
            const int b = u / M, m = u % M;
            PK_GLOBAL Cx<R> *Sr = out(b);
            if (!Sr) continue;
            PK_GLOBAL R *Sreal = (PK_GLOBAL R *)Sr;
            const Cx<R> zm = tile.at(b, m);
            if (m == 0) {
                const R X0 = zm.re + zm.im, XM = zm.re - zm.im;
                if constexpr (XW) {
                    Sreal[sine ? 2 * M - 1 : 0] = X0;
                    Sreal[sine ? M - 1 : M] = XM * w4[M].re;
                } else {
                    put(Sr, Cx<R>{X0, XM});
                }
            } else {
                Cx<R> xm, xc;
                split_pair(zm, tile.at(b, M - m), tw[m], xm, xc);
                if constexpr (XW)
                    wall_emit(Sreal, 2 * M, m, xm, w4, sine);  // C[m] and C[nx-m]
                else
                    put(Sr + m, xm);
            }
        }
    }
}

// Plain forward pass: x rows of f; optional per-workgroup sum of f.
// Persistent: workgroup w transforms the row blocks w, w + G, w + 2G, ...
// (G = gridDim.x) and loads the next block's pass-0 inputs into registers
// right after it has stored the current block's pass 0, so the HBM reads of
// block i+1 overlap the LDS passes and spectrum writes of block i.
template <int M, bool XW>
__global__ __launch_bounds__(XCfg<M>::NT) void k_x_fwd(XFwdArgs a0)
{
    if (gated_off(a0.batch, a0.gate, blockIdx.y)) return;
    XFwdArgs a = a0;
    if (a.batch) {
        const ProbPtrs &q = a.batch[blockIdx.y];
        a.f = q.f;
        a.S = q.S;
        if (a.partials) a.partials = q.partials;
    }
    using C = XCfg<M>;
    constexpr int NB = C::NB, NT = C::NT, NX = 2 * M;
    using Tile = LdsTile<R, M, NB, false, 0>;
    __shared__ Cx<R> s_tile[Tile::elems];
    __shared__ Cx<R> s_tw[NX];
    static_assert(sizeof(Cx<R>) * Tile::elems >= 3 * (NT / 64) * sizeof(double), "");

    const int nrows = a.ny * a.nz;
    const int nblk = (nrows + NB - 1) / NB;
    load_table(s_tw, (const Cx<R> *)a.tw, NX);

    double acc0 = 0.0;
    Tile tile{s_tile};
    PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
    const PK_GLOBAL double *gf = gbl(a.f);
    const bool sine = a.bc_x == 2;
    // walls: exp(-i pi k/(2nx)) in LDS for the cosine / sine read-out
    __shared__ Cx<R> s_w4[XW ? NX : 1];
    const Cx<R> *w4 = s_w4;
    if constexpr (XW) load_table(s_w4, (const Cx<R> *)a.tw4x, NX);
    auto loader = [&](int row0) {
        return [&, row0](int b, int n) -> Cx<R> {
            const int row = row0 + b;
            if (row >= nrows) return {R(0), R(0)};
            if constexpr (XW) {
                // walls: the reordered row v[j] = x[r(j)] (sines: signed)
                const int i0 = wall_index(2 * n, NX), i1 = wall_index(2 * n + 1, NX);
                double f0 = gf[(size_t)row * NX + i0], f1 = gf[(size_t)row * NX + i1];
                acc0 += (a.hz ? a.hz[row / a.ny] : 1.0) * (f0 + f1);
                if (sine) {
                    f0 = (i0 & 1) ? -f0 : f0;
                    f1 = (i1 & 1) ? -f1 : f1;
                }
                return {R(f0), R(f1)};
            } else {
            // f is read once (streaming loads measured 16 % faster for the
            // FP64 pass; the residual marches, which also read f, lost 1-3 %)
                const double2 fv = ld_stream(gf + (size_t)row * NX + 2 * n);
                // stretched z: the sum of f weighted by the plane thickness
                acc0 += (a.hz ? a.hz[row / a.ny] : 1.0) * (fv.x + fv.y);
                return {R(fv.x), R(fv.y)};
            }
        };
    };
    constexpr RPlan pl = make_rplan(M);
    if constexpr (XW) {
        // walls: contiguous row loads, stored reordered into the LDS tile
        // (x[2h] -> v[h], x[2h+1] -> v[nx-1-h], negated for sines), then
        // the transform from LDS
        for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
            const int row0 = block_order(blk, nblk, a.reverse) * NB;
            __syncthreads();  // tw table loaded / previous block done with the tile
            // all loads of the block in flight first, then the LDS stores
            constexpr int PERW = (NB * M + NT - 1) / NT;
            double2 fv[PERW];
#pragma unroll
            for (int q = 0; q < PERW; ++q) {
                const int e = threadIdx.x + q * NT;
                const int row = row0 + e / M;
                fv[q] = {0.0, 0.0};
                if (e < NB * M && row < nrows) fv[q] = ld_stream(gf + (size_t)row * NX + 2 * (e % M));
            }
#pragma unroll
            for (int q = 0; q < PERW; ++q) {
                const int e = threadIdx.x + q * NT;
                if (e >= NB * M) continue;
                const int b = e / M, h = e % M;
                acc0 += (a.hz ? a.hz[(row0 + b) / a.ny] : 1.0) * (fv[q].x + fv[q].y);
                R *trow = (R *)&tile.at(b, 0);
                trow[h] = R(fv[q].x);
                trow[NX - 1 - h] = R(sine ? -fv[q].y : fv[q].y);
            }
            __syncthreads();
            auto gload = [&](int b, int n) -> Cx<R> { return tile.at(b, n); };
            auto out = [&](int b) -> PK_GLOBAL Cx<R> * {
                const int row = row0 + b;
                return row < nrows ? S + (size_t)row * M : nullptr;
            };
            x_forward<M, NB, NT, true, 0, true>(s_tw, gload, tile, out, sine, w4);
        }
    } else if constexpr (pl.count >= 2) {
        Pass0Regs<R, M, NB, NT, false, 0, 0> in;
        int blk = blockIdx.x;
        if (blk < nblk) {
            auto gl = loader(block_order(blk, nblk, a.reverse) * NB);
            in.load(gl);
        }
        for (; blk < nblk; blk += gridDim.x) {
            const int row0 = block_order(blk, nblk, a.reverse) * NB;
            __syncthreads();  // tw table loaded / previous block done with the tile
            in.store(tile);
            const int nxt = blk + gridDim.x;
            if (nxt < nblk) {
                auto gl = loader(block_order(nxt, nblk, a.reverse) * NB);
                in.load(gl);
            }
            __syncthreads();
            auto out = [&](int b) -> PK_GLOBAL Cx<R> * {
                const int row = row0 + b;
                return row < nrows ? S + (size_t)row * M : nullptr;
            };
            auto gnone = [&](int, int) -> Cx<R> { return {R(0), R(0)}; };
            x_forward<M, NB, NT, false, 1, XW>(s_tw, gnone, tile, out, sine, w4);
        }
    } else {
        __syncthreads();
        for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
            const int row0 = block_order(blk, nblk, a.reverse) * NB;
            auto gl = loader(row0);
            auto out = [&](int b) -> PK_GLOBAL Cx<R> * {
                const int row = row0 + b;
                return row < nrows ? S + (size_t)row * M : nullptr;
            };
            x_forward<M, NB, NT, false, 0, XW>(s_tw, gl, tile, out, sine, w4);
            __syncthreads();
        }
    }

    if (a.partials) {
        // the reduction scratch reuses the tile once every wave is done with it
        double *s_red = (double *)s_tile;
        double z1 = 0.0, z2 = 0.0;
        __syncthreads();
        block_sum3(acc0, z1, z2, s_red);
        if (threadIdx.x == 0) {
            a.partials[4 * blockIdx.x] = acc0;
            a.partials[4 * blockIdx.x + 1] = 0.0;
            a.partials[4 * blockIdx.x + 2] = 0.0;
        }
    }
}

// Residual forward pass of the iterative refinement: the FP64 residual
// r = (f - mu) - L p of TJ y-rows is evaluated plane by plane with the 2.5-D
// march of stencil.hpp, rounded once to the transform precision, packed as
// z[h] = r[2h] + i r[2h+1] into the LDS tile (which aliases the march's plane
// tile) and transformed in place; per-workgroup FP64 sums of r^2,
// (f - mu)^2 and p go to `partials`.  r never touches HBM.  P32: p is the
// refinement's first iterate, read from its exact FP32 copy.  256 threads:
// with 512 the transform leaves threads idle and the pass is slower (237
// against 221 us at 512x512x256) although it runs four waves per SIMD
// instead of three.
constexpr int XR_NT = 256;

// One workgroup's work (plane range and row block vb.x of problem vb.y) of
// the residual pass; LDS carved from `lds` (LDS_BYTES).
template <int M, bool XW, bool P32> struct XRBody {
    static constexpr int TJ = march_rows_res(M), NT = XR_NT;
    using PT = typename std::conditional<P32, float, double>::type;
    using Mar = PlaneMarch<M, TJ, NT, PT>;
    using Tile = LdsTile<R, M, TJ, false, 0>;
    static constexpr size_t PLANE_B = sizeof(double2) * (TJ + 2) * M;
    static constexpr size_t FFT_B = sizeof(Cx<R>) * Tile::elems;
    static constexpr size_t BUF_B = ((PLANE_B > FFT_B ? PLANE_B : FFT_B) + 15) / 16 * 16;
    static constexpr size_t TW_B = sizeof(Cx<R>) * 2 * M;
    static constexpr size_t RED_B = (sizeof(double) * 3 * (NT / 64) + 15) / 16 * 16;
    static constexpr size_t LDS_BYTES = BUF_B + TW_B + RED_B + (XW ? TW_B : 0);

    static __device__ __forceinline__ void run(const XFwdArgs &a0, VBlock vb, char *lds)
    {

        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        XFwdArgs a = a0;
        if (a.batch) {
            const ProbPtrs &q = a.batch[vb.y];
            a.f = q.f;
            a.p = q.p;
            a.p32 = q.p32;
            a.S = q.S;
            a.partials = q.partials;
            a.sum_f = q.scal + 1;
        }
        constexpr int NX = 2 * M;
        char *s_buf = lds;
        Cx<R> *s_tw = (Cx<R> *)(lds + BUF_B);
        double *s_red = (double *)(lds + BUF_B + TW_B);

        const int njb = march_jblocks(a.ny, TJ);
        const int bid = block_order(xcd_order(vb.x, vb.gx), vb.gx, a.reverse);
        const int jb = bid % njb, kb = bid / njb;
        const int kr = march_planes(a.ny, a.nz, TJ, a.kr_max, a.kr_nb);
        const int k0 = kb * kr;
        const int k1 = k0 + kr < a.nz ? k0 + kr : a.nz;

        Mar m;
        m.f = gbl(a.f);
        if constexpr (P32)
            m.p = gbl(a.p32);
        else
            m.p = gbl(a.p);
        m.ax = a.ax;
        m.ay = a.ay;
        m.az = a.az;
        m.zc = a.zc;
        m.mu = (a.sum_f && !a.regular) ? (*a.sum_f) * a.inv_n : 0.0;
        m.tile = (double2(*)[M])s_buf;
        m.setup(jb, a.ny, a.nz, a.bc_z, a.bc_y);
        m.bc_x = XW ? a.bc_x : 0;
        const bool sine = a.bc_x == 2;
        Cx<R> *s_w4 = (Cx<R> *)(lds + BUF_B + TW_B + RED_B);
        const Cx<R> *w4 = s_w4;
        if constexpr (XW) load_table(s_w4, (const Cx<R> *)a.tw4x, NX, NT);
        load_table(s_tw, (const Cx<R> *)a.tw, NX, NT);
        m.start(k0);

        Tile tile{(Cx<R> *)s_buf};
        PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        for (int k = k0; k < k1; ++k) {
            __syncthreads();  // the previous plane's transform is done with the tile
            Cx<R> rr[Mar::PER];
            const double wk = a.hz ? a.hz[k] : 1.0;  // stretched z: volume weight of p
            auto sink = [&](int q, int, int, double r0, double r1, double f0, double f1, double2 c) {
                acc0 += r0 * r0 + r1 * r1;
                acc1 += f0 * f0 + f1 * f1;
                acc2 += wk * (c.x + c.y);
                rr[q] = {R(r0), R(r1)};
            };
            // loads of the next plane issued ahead of the transform (so that
            // they stay in flight during it) measured 6 % slower on MI355X
            m.fetch(k);
            m.step(k, sink);
            __syncthreads();  // the march is done reading the plane tile
#pragma unroll
            for (int q = 0; q < Mar::PER; ++q) {
                if (!m.valid(q)) continue;
                const int t = m.row_of(q), h = m.pair_of(q);
                if constexpr (XW) {
                    // walls: x[2h] -> v[h], x[2h+1] -> v[nx-1-h] (negated for sines)
                    R *trow = (R *)&tile.at(t, 0);
                    trow[h] = rr[q].re;
                    trow[NX - 1 - h] = sine ? -rr[q].im : rr[q].im;
                } else {
                    tile.at(t, h) = rr[q];
                }
            }
            __syncthreads();
            auto gload = [&](int b, int n) -> Cx<R> { return tile.at(b, n); };
            const size_t rowk = (size_t)k * a.ny + m.j0;
            const int V = m.V;
            auto out = [&](int b) -> PK_GLOBAL Cx<R> * { return b < V ? S + (rowk + b) * M : nullptr; };
            x_forward<M, TJ, NT, true, 0, XW>(s_tw, gload, tile, out, sine, w4);
        }
        block_sum3(acc0, acc1, acc2, s_red, NT);
        if (threadIdx.x == 0) {
            a.partials[4 * vb.x] = acc0;
            a.partials[4 * vb.x + 1] = acc1;
            a.partials[4 * vb.x + 2] = acc2;
        }
    }
};

template <int M, bool XW, bool P32>
__global__ __launch_bounds__(XR_NT) void k_x_res(XFwdArgs a0)
{
    using B = XRBody<M, XW, P32>;
    __shared__ __align__(16) char s_lds[B::LDS_BYTES];
    B::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, s_lds);
}

// Forward pass of the projection step: the right-hand side
// f = alpha D(u, v, w) (the divergence of the face velocities) of TJ y-rows
// is evaluated in FP64 plane by plane with the 2.5-D march of stencil.hpp,
// optionally stored (the refinement's residual passes read it), rounded once
// to the transform precision into the LDS tile (which aliases the march's
// staging arrays) and transformed in place; per-workgroup FP64 sums of f go
// to `partials` like those of the plain pass.  One problem per launch.
// Threads per workgroup: 512 with periodic x (at nx = 512 108 / 128 VGPRs
// in FP32 / FP64, four waves per SIMD; 441 / 394 against 455 / 402 us with
// 256 threads); the wall variants stay at 256 (with 512 they need more
// registers, not fewer).
template <bool XW> constexpr int xd_nt() { return XW ? 256 : 512; }

template <int M, bool XW>
__global__ __launch_bounds__(xd_nt<XW>()) void k_x_div(XFwdArgs a0)
{
    XFwdArgs a = a0;
    if (a.batch) {
        // the device-side loop passes its pointer records (one problem)
        const ProbPtrs &q = a.batch[0];
        a.S = q.S;
        if (a.partials) a.partials = q.partials;
    }
    constexpr int TJ = march_rows_res(M), NT = xd_nt<XW>(), NX = 2 * M;
    using Mar = DivMarch<M, TJ, NT>;
    using Tile = LdsTile<R, M, TJ, false, 0>;
    constexpr size_t PLANE_B = Mar::lds_bytes();
    constexpr size_t FFT_B = sizeof(Cx<R>) * Tile::elems;
    __shared__ __align__(16) char s_buf[PLANE_B > FFT_B ? PLANE_B : FFT_B];
    __shared__ Cx<R> s_tw[NX];
    __shared__ double s_red[3 * (NT / 64)];

    const int njb = march_jblocks(a.ny, TJ);
    const int bid = xcd_order(blockIdx.x, gridDim.x);
    const int jb = bid % njb, kb = bid / njb;
    const int kr = march_planes(a.ny, a.nz, TJ, a.kr_max, a.kr_nb);
    const int k0 = kb * kr;
    const int k1 = k0 + kr < a.nz ? k0 + kr : a.nz;

    Mar m;
    m.u = gbl(a.u);
    m.v = gbl(a.v);
    m.w = gbl(a.w);
    m.cx = a.cx;
    m.cy = a.cy;
    m.cz = a.cz;
    m.xwall = a.bc_x != 0;
    m.ywall = a.bc_y != 0;
    m.bind(s_buf);
    m.setup(jb, a.ny, a.nz, a.bc_z);
    load_table(s_tw, (const Cx<R> *)a.tw, NX);
    // walls along x: cosine expansion of the rows (exp(-i pi k/(2nx)) in LDS)
    __shared__ Cx<R> s_w4[XW ? NX : 1];
    if constexpr (XW) load_table(s_w4, (const Cx<R> *)a.tw4x, NX);
    const bool sine = a.bc_x == 2;
    m.start(k0);

    Tile tile{(Cx<R> *)s_buf};
    PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
    PK_GLOBAL double *fo = a.f_out ? gbl(a.f_out) : nullptr;
    double acc0 = 0.0;
    for (int k = k0; k < k1; ++k) {
        __syncthreads();  // the previous plane's transform is done with the tile
        Cx<R> ff[Mar::PER];
        const size_t kp = (size_t)k * m.plane;
        auto sink = [&](int q, int, int, double f0, double f1) {
            acc0 += f0 + f1;
            ff[q] = {R(f0), R(f1)};
            if (fo) *(PK_GLOBAL double2 *)(fo + kp + m.roff(q)) = double2{f0, f1};
        };
        m.step(k, sink);
        __syncthreads();  // the march is done reading its staging arrays
#pragma unroll
        for (int q = 0; q < Mar::PER; ++q) {
            if (!m.valid(q)) continue;
            const int t = m.row_of(q), h = m.pair_of(q);
            if constexpr (XW) {
                // x[2h] -> v[h], x[2h+1] -> v[nx-1-h]
                R *trow = (R *)&tile.at(t, 0);
                trow[h] = ff[q].re;
                trow[NX - 1 - h] = sine ? -ff[q].im : ff[q].im;
            } else {
                tile.at(t, h) = ff[q];
            }
        }
        __syncthreads();
        auto gload = [&](int b, int n) -> Cx<R> { return tile.at(b, n); };
        const size_t rowk = (size_t)k * a.ny + m.j0;
        const int V = m.V;
        auto out = [&](int b) -> PK_GLOBAL Cx<R> * { return b < V ? S + (rowk + b) * M : nullptr; };
        x_forward<M, TJ, NT, true, 0, XW>(s_tw, gload, tile, out, sine, s_w4);
    }
    if (a.partials) {
        double z1 = 0.0, z2 = 0.0;
        block_sum3(acc0, z1, z2, s_red);
        if (threadIdx.x == 0) {
            a.partials[4 * blockIdx.x] = acc0;
            a.partials[4 * blockIdx.x + 1] = 0.0;
            a.partials[4 * blockIdx.x + 2] = 0.0;
        }
    }
}

// One workgroup's work (row block vb.x of problem vb.y) of the inverse pass;
// LDS carved from `lds` (LDS_BYTES).
template <int M, bool ACC, bool XW, bool P32> struct XIBody {
    using C = XCfg<M>;
    using Tile = LdsTile<R, M, C::NB, false, C::PAD>;
    static constexpr size_t TILE_B = sizeof(Cx<R>) * Tile::elems;
    static constexpr size_t LDS_BYTES = TILE_B + sizeof(Cx<R>) * 2 * M;

    static __device__ __forceinline__ void run(const XInvArgs &a0, VBlock vb, char *lds)
    {

        // P32: the first iterate lives in FP32 (a.p32); the plain pass writes it
        // there, the accumulating pass reads it there and writes p.  A problem
        // of the device-side loop that stopped before any correction (C_COPY)
        // gets p = p32 widened instead.
        bool widen_only = false;
        if constexpr (P32 && ACC) {
            if (a0.batch && a0.gate) {
                const int *c = a0.batch[vb.y].ctrl;
                if (c[C_CORRECT] == 0) {
                    if (c[C_COPY] == 0) return;
                    widen_only = true;
                }
            }
        } else {
            if (gated_off(a0.batch, a0.gate, vb.y)) return;
        }
        XInvArgs a = a0;
        if (a.batch) {
            const ProbPtrs &q = a.batch[vb.y];
            a.S = q.S;
            a.p = q.p;
            a.p32 = q.p32;
            if (ACC && a.sum_p) a.sum_p = q.scal + 4;
        }
        // accumulate mode also removes the mean of the previous iterate (the
        // residual cannot see the constant mode, so the gauge is kept here)
        const double pmean = (ACC && a.sum_p && !a.regular) ? (*a.sum_p) * a.inv_n : 0.0;
        constexpr int NB = C::NB, NT = C::NT, NX = 2 * M;
        Cx<R> *s_tile = (Cx<R> *)lds;
        Cx<R> *s_tw = (Cx<R> *)(lds + TILE_B);

        const int nrows = a.ny * a.nz;
        const int row0 = block_order(vb.x, vb.gx, a.reverse) * NB;
        PK_GLOBAL double *gp = gbl(a.p);
        PK_GLOBAL float *gp32 = gbl(a.p32);
        if (widen_only) {  // uniform over the workgroup
            for (int e = threadIdx.x; e < NB * M; e += NT) {
                const int row = row0 + e / M;
                if (row >= nrows) break;
                const size_t o = (size_t)row * NX + 2 * (e % M);
                st_stream(gp + o, ld_stream(gp32 + o));
            }
            return;
        }
        load_table(s_tw, (const Cx<R> *)a.tw, NX, NT);
        __syncthreads();

        const PK_GLOBAL Cx<R> *S = gbl((const Cx<R> *)a.S);
        const bool sine = a.bc_x == 2;
        const PK_GLOBAL Cx<R> *w4 = XW ? gbl((const Cx<R> *)a.tw4x) : nullptr;
        auto gstore = [&](int b, int n, Cx<R> v) {
            const int row = row0 + b;
            if (row >= nrows) return;
            double2 o = {double(v.re), -double(v.im)};
            if constexpr (XW) {
                // walls: v[j] goes back to x[r(j)] (negated at odd x for sines)
                const int i0 = wall_index(2 * n, NX), i1 = wall_index(2 * n + 1, NX);
                if (sine) {
                    o.x = (i0 & 1) ? -o.x : o.x;
                    o.y = (i1 & 1) ? -o.y : o.y;
                }
                PK_GLOBAL double *rp = gp + (size_t)row * NX;
                PK_GLOBAL float *rp32 = gp32 + (size_t)row * NX;
                if constexpr (ACC) {
                    o.x += (P32 ? (double)rp32[i0] : rp[i0]) - pmean;
                    o.y += (P32 ? (double)rp32[i1] : rp[i1]) - pmean;
                }
                if constexpr (P32 && !ACC) {
                    rp32[i0] = (float)o.x;
                    rp32[i1] = (float)o.y;
                } else {
                    rp[i0] = o.x;
                    rp[i1] = o.y;
                }
                return;
            }
            const size_t di = (size_t)row * NX + 2 * n;
            if constexpr (ACC) {
                const double2 old = P32 ? ld_stream(gp32 + di) : ld_stream(gp + di);
                o.x += old.x - pmean;
                o.y += old.y - pmean;
            }
            if constexpr (P32 && !ACC)
                st_stream(gp32 + di, o);
            else
                st_stream(gp + di, o);
        };
        // spectrum value m of a row: the packed half spectrum, or for walls the
        // inverse input formed from the cosine / sine coefficients
        auto xval = [&](const PK_GLOBAL Cx<R> *sr, int m) -> Cx<R> {
            if constexpr (XW)
                return wall_load((const PK_GLOBAL R *)sr, NX, m, w4, sine);
            else
                return sr[m];
        };
        // reversed radix order: the small radix first gives more butterfly pairs
        // per row for the fused first pass
        constexpr RPlan pl = get_rplan(M, 1);
        // Accumulating, the previous iterate's values of the block are loaded
        // before the transform (with the fused first pass), in the coalesced
        // order of the final store loop, so that their reads are in flight
        // during it; the last pass stores into the tile and the loop adds and
        // writes p.  Loaded in the last pass's stores (periodic x) or after
        // the transform (walls), their latency was exposed.
        constexpr bool PRE = ACC && pl.count >= 2 && (M / pl.r[0]) % 2 == 0;
        constexpr int PERP = PRE ? (NB * M + NT - 1) / NT : 1;
        using PV2 = typename std::conditional<P32, pk_f2v, pk_d2v>::type;
        Tile tile{s_tile};
        // walls: the tile holds conj(v) of each row in transform order; write
        // x[2h] = v[h], x[2h+1] = v[nx-1-h] (negated for sines) with contiguous
        // stores (or accumulate)
        auto wall_rows_out = [&](const auto &pre) {
            __syncthreads();
            constexpr int PERW = (NB * M + NT - 1) / NT;
            double2 old[PERW];
            if constexpr (PRE) {  // loaded before the transform
                static_assert(PERW == PERP, "same coalesced order");
#pragma unroll
                for (int q = 0; q < PERW; ++q) old[q] = {double(pre[q].x), double(pre[q].y)};
            } else if constexpr (ACC) {
                // all loads of the previous iterate in flight first
#pragma unroll
                for (int q = 0; q < PERW; ++q) {
                    const int e = threadIdx.x + q * NT;
                    const int row = row0 + e / M;
                    old[q] = {0.0, 0.0};
                    if (e < NB * M && row < nrows) {
                        const size_t oi = (size_t)row * NX + 2 * (e % M);
                        old[q] = P32 ? ld_stream(gp32 + oi) : ld_stream(gp + oi);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < PERW; ++q) {
                const int e = threadIdx.x + q * NT;
                const int b = e / M, h = e % M;
                const int row = row0 + b;
                if (e >= NB * M || row >= nrows) continue;
                const R *trow = (const R *)&tile.at(b, 0);
                // the tile holds conj(z), z[j] = v[2j] + i v[2j+1]
                const int j1 = NX - 1 - h;
                const double v0 = (h & 1) ? -double(trow[h]) : double(trow[h]);
                double v1 = (j1 & 1) ? -double(trow[j1]) : double(trow[j1]);
                if (sine) v1 = -v1;
                double2 o = {v0, v1};
                if constexpr (ACC) {
                    o.x += old[q].x - pmean;
                    o.y += old[q].y - pmean;
                }
                if constexpr (P32 && !ACC)
                    st_stream(gp32 + (size_t)row * NX + 2 * h, o);
                else
                    st_stream(gp + (size_t)row * NX + 2 * h, o);
            }
        };
        PV2 pre[PERP];
        if constexpr (PRE) {
#pragma unroll
            for (int q = 0; q < PERP; ++q) {
                const int e = threadIdx.x + q * NT;
                const int row = row0 + e / M;
                pre[q] = PV2{0, 0};
                if ((NB * M) % NT == 0 || e < NB * M)
                    if (row < nrows) {
                        const size_t o = (size_t)row * NX + 2 * (e % M);
                        if constexpr (P32)
                            pre[q] = __builtin_nontemporal_load((const PK_GLOBAL pk_f2v *)(gp32 + o));
                        else
                            pre[q] = __builtin_nontemporal_load((const PK_GLOBAL pk_d2v *)(gp + o));
                    }
            }
        }
        if constexpr (pl.count >= 2 && (M / pl.r[0]) % 2 == 0) {
            // first pass with the merge fused (no twiddles in a first pass),
            // outputs of butterfly j to the LDS tile at j RAD + r
            constexpr int RAD = pl.r[0];
            constexpr int NJ = M / RAD;
            static_assert(NJ % 2 == 0, "pairing needs even NJ");
            constexpr int U = NJ / 2, NU = NB * U;
            constexpr int PER = (NU + NT - 1) / NT;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u / U, pp = u % U;
                int j1, j2;
                pair_of<NJ>(pp, j1, j2);
                const int row = row0 + b;
                Cx<R> v1[RAD], v2[RAD];
                if (row < nrows) {
                    const PK_GLOBAL Cx<R> *sr = S + (size_t)row * M;
#pragma unroll
                    for (int r = 0; r < RAD; ++r) {
                        v1[r] = xval(sr, j1 + r * NJ);
                        v2[r] = xval(sr, j2 + r * NJ);
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < RAD; ++r) v1[r] = v2[r] = {R(0), R(0)};
                }
                Cx<R> z1[RAD], z2[RAD];
                if (pp == 0) {
                    // m = 0 unpacks X(0) + i X(M); butterfly 0 pairs r <-> RAD-r
                    z1[0] = {v1[0].re + v1[0].im, -(v1[0].re - v1[0].im)};
#pragma unroll
                    for (int r = 1; r < RAD; ++r)
                        if (r <= RAD - r) merge_pair(v1[r], v1[RAD - r], s_tw[r * NJ], z1[r], z1[RAD - r]);
#pragma unroll
                    for (int r = 0; r < RAD; ++r)
                        if (r <= RAD - 1 - r)
                            merge_pair(v2[r], v2[RAD - 1 - r], s_tw[NJ / 2 + r * NJ], z2[r],
                                       z2[RAD - 1 - r]);
                } else {
#pragma unroll
                    for (int r = 0; r < RAD; ++r)
                        merge_pair(v1[r], v2[RAD - 1 - r], s_tw[j1 + r * NJ], z1[r], z2[RAD - 1 - r]);
                }
                Bfly<R, RAD>::run(z1);
                Bfly<R, RAD>::run(z2);
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    tile.at(b, j1 * RAD + r) = z1[r];
                    tile.at(b, j2 * RAD + r) = z2[r];
                }
            }
            __syncthreads();
            auto gnone = [&](int, int) -> Cx<R> { return {R(0), R(0)}; };
            if constexpr (XW) {
                // the last pass stores back into the tile (it synchronises between
                // its reads and writes); rows are then written contiguously
                auto tstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
                fft_passes<R, M, NB, NT, false, C::PAD, false, 1, pl.count, 1>(s_tw, 2, gnone,
                                                                               tstore, tile);
                wall_rows_out(pre);
            } else if constexpr (PRE) {
                auto tstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
                fft_passes<R, M, NB, NT, false, C::PAD, false, 1, pl.count, 1>(s_tw, 2, gnone,
                                                                               tstore, tile);
                __syncthreads();
#pragma unroll
                for (int q = 0; q < PERP; ++q) {
                    const int e = threadIdx.x + q * NT;
                    const int b = e / M, h = e % M;
                    const int row = row0 + b;
                    if (((NB * M) % NT != 0 && e >= NB * M) || row >= nrows) continue;
                    const Cx<R> v = tile.at(b, h);
                    const double2 o = {double(v.re) + (double(pre[q].x) - pmean),
                                       -double(v.im) + (double(pre[q].y) - pmean)};
                    st_stream(gp + (size_t)row * NX + 2 * h, o);
                }
            } else {
                fft_passes<R, M, NB, NT, false, C::PAD, false, 1, pl.count, 1>(s_tw, 2, gnone,
                                                                               gstore, tile);
            }
        } else {
            auto gload = [&](int b, int n) -> Cx<R> {
                const int row = row0 + b;
                if (row >= nrows) return {R(0), R(0)};
                const PK_GLOBAL Cx<R> *sr = S + (size_t)row * M;
                if (n == 0) {
                    const Cx<R> s0 = xval(sr, 0);
                    return {s0.re + s0.im, -(s0.re - s0.im)};
                }
                Cx<R> zm, zc;
                merge_pair(xval(sr, n), xval(sr, M - n), s_tw[n], zm, zc);
                return zm;
            };
            if constexpr (XW) {
                auto tstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
                fft_tile<R, M, NB, NT, false, C::PAD, false>(s_tw, 2, gload, tstore, tile);
                wall_rows_out(pre);
            } else {
                fft_tile<R, M, NB, NT, false, C::PAD, false>(s_tw, 2, gload, gstore, tile);
            }
        }
    }
};

template <int M, bool ACC, bool XW, bool P32>
__global__ __launch_bounds__(XCfg<M>::NT) void k_x_inv(XInvArgs a0)
{
    using B = XIBody<M, ACC, XW, P32>;
    __shared__ __align__(16) char s_lds[B::LDS_BYTES];
    B::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, s_lds);
}

// row blocks of the plain pass (an upper bound of its workgroup count), or
// the workgroups of the residual pass
template <int M> static int blocks_x(int ny, int nz, int residual, int kr_max, int kr_nb)
{
    if (residual)  // residual and divergence passes: the same plane march
        return march_jblocks(ny, march_rows_res(M)) *
               march_kblocks(ny, nz, march_rows_res(M), kr_max, kr_nb);
    return (ny * nz + XCfg<M>::NB - 1) / XCfg<M>::NB;
}

// workgroups of the persistent plain pass: as many as are resident on the
// device at once (shared among the problems of a batched launch)
template <int M, bool XW> static int grid_x_fwd(int nblk, int nbatch)
{
    static int resident[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    int &r = resident[dev & 63];
    if (r == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_x_fwd<M, XW>, XCfg<M>::NT, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1) {
            (void)hipGetLastError();
            per_cu = 1;
            cus = 256;
        }
        r = per_cu * cus;
    }
    int g = r / (nbatch > 0 ? nbatch : 1);
    g = g < 1 ? 1 : g;
    return g < nblk ? g : nblk;
}

template <int M> static int run_x_fwd(const XFwdArgs &a, hipStream_t s, int *nblocks_out)
{
    const bool xw = a.bc_x != 0;
    int nb = blocks_x<M>(a.ny, a.nz, a.residual, a.kr_max, a.kr_nb);
    if (!a.residual) nb = xw ? grid_x_fwd<M, true>(nb, a.batch ? a.nbatch : 1)
                             : grid_x_fwd<M, false>(nb, a.batch ? a.nbatch : 1);
    if (nblocks_out) *nblocks_out = nb;
    const dim3 grid(nb, a.batch ? a.nbatch : 1);
    if (a.residual == 2) {
        if (a.batch && a.nbatch != 1) return -1;
        if (xw)
            hipLaunchKernelGGL((k_x_div<M, true>), dim3(nb), dim3(xd_nt<true>()), 0, s, a);
        else
            hipLaunchKernelGGL((k_x_div<M, false>), dim3(nb), dim3(xd_nt<false>()), 0, s, a);
    } else if (a.residual) {
        // the refinement transforms its residual in FP32 only
        if constexpr (sizeof(R) == 4) {
            if (a.p_in32) {
                if (xw)
                    hipLaunchKernelGGL((k_x_res<M, true, true>), grid, dim3(XR_NT), 0, s, a);
                else
                    hipLaunchKernelGGL((k_x_res<M, false, true>), grid, dim3(XR_NT), 0, s,
                                       a);
            } else if (xw) {
                hipLaunchKernelGGL((k_x_res<M, true, false>), grid, dim3(XR_NT), 0, s, a);
            } else {
                hipLaunchKernelGGL((k_x_res<M, false, false>), grid, dim3(XR_NT), 0, s, a);
            }
        } else {
            return -1;
        }
    } else if (xw) {
        hipLaunchKernelGGL((k_x_fwd<M, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_x_fwd<M, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
    }
    return (int)hipGetLastError();
}

template <int M> static int run_x_inv(const XInvArgs &a, hipStream_t s)
{
    const int nrows = a.ny * a.nz;
    const int nb = (nrows + XCfg<M>::NB - 1) / XCfg<M>::NB;
    const dim3 grid(nb, a.batch ? a.nbatch : 1);
    const bool xw = a.bc_x != 0;
    if (a.p_in32) {
        // the refinement keeps its first iterate in FP32 only
        if constexpr (sizeof(R) == 4) {
            if (a.accumulate) {
                if (xw)
                    hipLaunchKernelGGL((k_x_inv<M, true, true, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
                else
                    hipLaunchKernelGGL((k_x_inv<M, true, false, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
            } else {
                if (xw)
                    hipLaunchKernelGGL((k_x_inv<M, false, true, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
                else
                    hipLaunchKernelGGL((k_x_inv<M, false, false, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
            }
        } else {
            return -1;
        }
    } else if (a.accumulate) {
        if (xw)
            hipLaunchKernelGGL((k_x_inv<M, true, true, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_x_inv<M, true, false, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
    } else {
        if (xw)
            hipLaunchKernelGGL((k_x_inv<M, false, true, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_x_inv<M, false, false, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
    }
    return (int)hipGetLastError();
}


}  // namespace PK_NS
using namespace PK_NS;

// the host launchers are defined once, in this file's own object (the
// work-list source includes this file for its kernel bodies)
#ifndef PK_X_LIST_TU
#define PK_CASE_FWD(N) case N: return run_x_fwd<N>(a, s, nblocks_out);
#define PK_CASE_INV(N) case N: return run_x_inv<N>(a, s);
#define PK_CASE_BLK(N) case N: return blocks_x<N>(ny, nz, residual, kr_max, kr_nb);

int PK_SUFFIX(launch_x_fwd)(const XFwdArgs &a, hipStream_t s, int *nblocks_out)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_FWD) default: return -1; }
}

int PK_SUFFIX(launch_x_inv)(const XInvArgs &a, hipStream_t s)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_INV) default: return -1; }
}

int PK_SUFFIX(x_fwd_blocks)(int nx, int ny, int nz, int residual, int kr_max, int kr_nb)
{
    switch (nx / 2) { PK_X_LENGTHS(PK_CASE_BLK) default: return -1; }
}

// workgroups (partial records) launch_x_fwd uses for this record
template <int M> static int grid_of(const XFwdArgs &a)
{
    int nb = blocks_x<M>(a.ny, a.nz, a.residual, a.kr_max, a.kr_nb);
    if (!a.residual)
        nb = a.bc_x != 0 ? grid_x_fwd<M, true>(nb, a.batch ? a.nbatch : 1)
                         : grid_x_fwd<M, false>(nb, a.batch ? a.nbatch : 1);
    return nb;
}
#define PK_CASE_GRID(N) case N: return grid_of<N>(a);

int PK_SUFFIX(x_fwd_grid)(const XFwdArgs &a)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_GRID) default: return -1; }
}

// resident workgroups of the residual pass with transform on the current
// device (FP32 transform only)
template <int M, bool XW, bool P32> static int res_slots()
{
    if constexpr (sizeof(R) != 4) {
        return -1;
    } else {
        static int cache[64] = {0};
        int dev = 0;
        (void)hipGetDevice(&dev);
        int &r = cache[dev & 63];
        if (r == 0) {
            int per_cu = 0, cus = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_x_res<M, XW, P32>, XR_NT,
                                                             0) != hipSuccess ||
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                    hipSuccess ||
                per_cu < 1 || cus < 1) {
                (void)hipGetLastError();
                return -1;
            }
            r = per_cu * cus;
        }
        return r;
    }
}
template <int M> static int res_slots_of(int xw, int p32)
{
    return xw ? (p32 ? res_slots<M, true, true>() : res_slots<M, true, false>())
              : (p32 ? res_slots<M, false, true>() : res_slots<M, false, false>());
}
#define PK_CASE_SLOTS(N) case N: return res_slots_of<N>(xw, p32);

int PK_SUFFIX(x_res_slots)(int nx, int xw, int p32)
{
    switch (nx / 2) { PK_X_LENGTHS(PK_CASE_SLOTS) default: return -1; }
}
#endif

}  // namespace pk
