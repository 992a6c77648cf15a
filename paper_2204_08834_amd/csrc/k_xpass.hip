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
// iterative refinement, evaluated from f and p as the row is loaded (its L2
// norm and that of f - mu accumulate in FP64 per workgroup), so r never
// touches HBM.
//
// Inverse: Z'[m] = (X[m] + conj X[M-m]) + i w^-m (X[m] - conj X[M-m]) with
// Z'[0] = (X[0] + X[M]) + i (X[0] - X[M]); an inverse M-point FFT of Z'
// returns nx (x[2n] + i x[2n+1]) (unnormalised, like the forward pass), which
// is stored to p or added to it in FP64.
//
// Compiled once per precision with PK_REAL = float or double.
#include "fft_core.hpp"
#include "lengths.hpp"

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

// sum three doubles over the workgroup; thread 0 gets the totals
__device__ __forceinline__ void block_sum3(double &a, double &b, double &c, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
        c += __shfl_down(c, off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) { sh[3 * wid] = a; sh[3 * wid + 1] = b; sh[3 * wid + 2] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        a = 0.0;
        b = 0.0;
        c = 0.0;
        for (int w = 0; w < nw; ++w) { a += sh[3 * w]; b += sh[3 * w + 1]; c += sh[3 * w + 2]; }
    }
}

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

template <int M, bool RES>
__global__ __launch_bounds__(XCfg<M>::NT) void k_x_fwd(XFwdArgs a0)
{
    XFwdArgs a = a0;
    if (a.batch) {
        const ProbPtrs &q = a.batch[blockIdx.y];
        a.f = q.f;
        a.p = q.p;
        a.S = q.S;
        if (a.partials) a.partials = q.partials;
        a.sum_f = q.scal + 1;
    }
    using C = XCfg<M>;
    constexpr int NB = C::NB, NT = C::NT, NX = 2 * M;
    using Tile = LdsTile<R, M, NB, false, C::PAD>;
    __shared__ Cx<R> s_tile[Tile::elems];
    __shared__ Cx<R> s_tw[NX];
    static_assert(sizeof(Cx<R>) * Tile::elems >= 3 * (NT / 64) * sizeof(double), "");

    const int nrows = a.ny * a.nz;
    const int row0 = block_order(blockIdx.x, gridDim.x, a.reverse) * NB;
    load_table(s_tw, (const Cx<R> *)a.tw, NX);
    __syncthreads();

    const double mu = (RES && a.sum_f) ? (*a.sum_f) * a.inv_n : 0.0;
    // plain input: acc0 = sum f; residual: sum r^2, sum (f - mu)^2, sum p
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    auto gload = [&](int b, int n) -> Cx<R> {
        const int row = row0 + b;
        if (row >= nrows) return {R(0), R(0)};
        const size_t roff = (size_t)row * NX;
        const double2 fv = *(const double2 *)(a.f + roff + 2 * n);
        if constexpr (!RES) {
            acc0 += fv.x + fv.y;
            return {R(fv.x), R(fv.y)};
        }
        const int j = row % a.ny, k = row / a.ny;
        const double *pr = a.p + roff;
        const double2 pc = *(const double2 *)(pr + 2 * n);
        const double pl = pr[(2 * n + NX - 1) % NX];
        const double pq = pr[(2 * n + 2) % NX];
        const int jm = (j == 0) ? a.ny - 1 : j - 1;
        const int jp = (j == a.ny - 1) ? 0 : j + 1;
        int km, kp;
        if (a.bc_z == 0) {
            km = (k == 0) ? a.nz - 1 : k - 1;
            kp = (k == a.nz - 1) ? 0 : k + 1;
        } else {  // mirrored ghost at the walls
            km = (k == 0) ? 0 : k - 1;
            kp = (k == a.nz - 1) ? k : k + 1;
        }
        const size_t plane = (size_t)a.ny * NX;
        const double2 ps = *(const double2 *)(a.p + (size_t)k * plane + (size_t)jm * NX + 2 * n);
        const double2 pn = *(const double2 *)(a.p + (size_t)k * plane + (size_t)jp * NX + 2 * n);
        const double2 pd = *(const double2 *)(a.p + (size_t)km * plane + (size_t)j * NX + 2 * n);
        const double2 pu = *(const double2 *)(a.p + (size_t)kp * plane + (size_t)j * NX + 2 * n);
        const double l0 = a.ax * (pc.y - 2.0 * pc.x + pl) + a.ay * (pn.x - 2.0 * pc.x + ps.x) +
                          a.az * (pu.x - 2.0 * pc.x + pd.x);
        const double l1 = a.ax * (pq - 2.0 * pc.y + pc.x) + a.ay * (pn.y - 2.0 * pc.y + ps.y) +
                          a.az * (pu.y - 2.0 * pc.y + pd.y);
        const double f0 = fv.x - mu, f1 = fv.y - mu;
        const double r0 = f0 - l0, r1 = f1 - l1;
        acc0 += r0 * r0 + r1 * r1;
        acc1 += f0 * f0 + f1 * f1;
        acc2 += pc.x + pc.y;
        return {R(r0), R(r1)};
    };
    Tile tile{s_tile};
    auto lstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
    Cx<R> *S = (Cx<R> *)a.S;
    constexpr RPlan pl = make_rplan(M);
    if constexpr (pl.count >= 2) {
        // all passes but the last, then the last pass with the split fused
        fft_passes<R, M, NB, NT, false, C::PAD, false, 0, pl.count - 1, 0>(s_tw, 2, gload, lstore,
                                                                           tile);
        __syncthreads();
        constexpr int RAD = pl.r[pl.count - 1];
        constexpr int NJ = M / RAD;
        static_assert(NJ == rplan_ns(pl, pl.count - 1) && NJ % 2 == 0, "pairing needs even NJ");
        constexpr int U = NJ / 2, NU = NB * U;
        constexpr int PER = (NU + NT - 1) / NT;
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
                v1[r] = cmul(v1[r], s_tw[2 * r * j1]);
                v2[r] = cmul(v2[r], s_tw[2 * r * j2]);
            }
            Bfly<R, RAD>::run(v1);
            Bfly<R, RAD>::run(v2);
            const int row = row0 + b;
            if (row >= nrows) continue;
            Cx<R> *Sr = S + (size_t)row * M;
            auto emit = [&](int m, Cx<R> zm, Cx<R> zc) {
                Cx<R> xm, xc;
                split_pair(zm, zc, s_tw[m], xm, xc);
                Sr[m] = xm;
                if (2 * m != M) Sr[M - m] = xc;
            };
            if (pp == 0) {
                // butterfly 0: m = r NJ; m = 0 packs X(0) + i X(M)
                Sr[0] = {v1[0].re + v1[0].im, v1[0].re - v1[0].im};
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
    } else {
        fft_tile<R, M, NB, NT, false, C::PAD, false>(s_tw, 2, gload, lstore, tile);
        __syncthreads();
        // split the M-point spectrum into the half spectrum of the real rows
        for (int u = threadIdx.x; u < NB * M; u += NT) {
            const int b = u / M, m = u % M;
            const int row = row0 + b;
            if (row >= nrows) continue;
            const Cx<R> zm = tile.at(b, m);
            if (m == 0) {
                S[(size_t)row * M] = {zm.re + zm.im, zm.re - zm.im};
            } else {
                Cx<R> xm, xc;
                split_pair(zm, tile.at(b, M - m), s_tw[m], xm, xc);
                S[(size_t)row * M + m] = xm;
            }
        }
    }

    if (a.partials) {
        // the reduction scratch reuses the tile once every wave is done with it
        double *s_red = (double *)s_tile;
        __syncthreads();
        block_sum3(acc0, acc1, acc2, s_red);
        if (threadIdx.x == 0) {
            a.partials[4 * blockIdx.x] = acc0;
            a.partials[4 * blockIdx.x + 1] = acc1;
            a.partials[4 * blockIdx.x + 2] = acc2;
        }
    }
}

template <int M, bool ACC>
__global__ __launch_bounds__(XCfg<M>::NT) void k_x_inv(XInvArgs a0)
{
    XInvArgs a = a0;
    if (a.batch) {
        const ProbPtrs &q = a.batch[blockIdx.y];
        a.S = q.S;
        a.p = q.p;
        if (ACC && a.sum_p) a.sum_p = q.scal + 4;
    }
    // accumulate mode also removes the mean of the previous iterate (the
    // residual cannot see the constant mode, so the gauge is kept here)
    const double pmean = (ACC && a.sum_p) ? (*a.sum_p) * a.inv_n : 0.0;
    using C = XCfg<M>;
    constexpr int NB = C::NB, NT = C::NT, NX = 2 * M;
    using Tile = LdsTile<R, M, NB, false, C::PAD>;
    __shared__ Cx<R> s_tile[Tile::elems];
    __shared__ Cx<R> s_tw[NX];

    const int nrows = a.ny * a.nz;
    const int row0 = block_order(blockIdx.x, gridDim.x, a.reverse) * NB;
    load_table(s_tw, (const Cx<R> *)a.tw, NX);
    __syncthreads();

    const Cx<R> *S = (const Cx<R> *)a.S;
    auto gstore = [&](int b, int n, Cx<R> v) {
        const int row = row0 + b;
        if (row >= nrows) return;
        double2 *dst = (double2 *)(a.p + (size_t)row * NX + 2 * n);
        double2 o = {double(v.re), -double(v.im)};
        if constexpr (ACC) {
            const double2 old = *dst;
            o.x += old.x - pmean;
            o.y += old.y - pmean;
        }
        *dst = o;
    };
    Tile tile{s_tile};
    // reversed radix order: the small radix first gives more butterfly pairs
    // per row for the fused first pass
    constexpr RPlan pl = get_rplan(M, 1);
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
                const Cx<R> *sr = S + (size_t)row * M;
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    v1[r] = sr[j1 + r * NJ];
                    v2[r] = sr[j2 + r * NJ];
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
        fft_passes<R, M, NB, NT, false, C::PAD, false, 1, pl.count, 1>(s_tw, 2, gnone, gstore,
                                                                       tile);
    } else {
        auto gload = [&](int b, int n) -> Cx<R> {
            const int row = row0 + b;
            if (row >= nrows) return {R(0), R(0)};
            const Cx<R> *sr = S + (size_t)row * M;
            if (n == 0) {
                const Cx<R> s0 = sr[0];
                return {s0.re + s0.im, -(s0.re - s0.im)};
            }
            Cx<R> zm, zc;
            merge_pair(sr[n], sr[M - n], s_tw[n], zm, zc);
            return zm;
        };
        fft_tile<R, M, NB, NT, false, C::PAD, false>(s_tw, 2, gload, gstore, tile);
    }
}

template <int M> static int run_x_fwd(const XFwdArgs &a, hipStream_t s)
{
    const int nrows = a.ny * a.nz;
    const int nb = (nrows + XCfg<M>::NB - 1) / XCfg<M>::NB;
    const dim3 grid(nb, a.batch ? a.nbatch : 1);
    if (a.residual)
        hipLaunchKernelGGL((k_x_fwd<M, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_x_fwd<M, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
    return (int)hipGetLastError();
}

template <int M> static int run_x_inv(const XInvArgs &a, hipStream_t s)
{
    const int nrows = a.ny * a.nz;
    const int nb = (nrows + XCfg<M>::NB - 1) / XCfg<M>::NB;
    const dim3 grid(nb, a.batch ? a.nbatch : 1);
    if (a.accumulate)
        hipLaunchKernelGGL((k_x_inv<M, true>), grid, dim3(XCfg<M>::NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_x_inv<M, false>), grid, dim3(XCfg<M>::NT), 0, s, a);
    return (int)hipGetLastError();
}

template <int M> static int blocks_x(int ny, int nz)
{
    return (ny * nz + XCfg<M>::NB - 1) / XCfg<M>::NB;
}

}  // namespace PK_NS
using namespace PK_NS;

#define PK_CASE_FWD(N) case N: return run_x_fwd<N>(a, s);
#define PK_CASE_INV(N) case N: return run_x_inv<N>(a, s);
#define PK_CASE_BLK(N) case N: return blocks_x<N>(ny, nz);

int PK_SUFFIX(launch_x_fwd)(const XFwdArgs &a, hipStream_t s)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_FWD) default: return -1; }
}

int PK_SUFFIX(launch_x_inv)(const XInvArgs &a, hipStream_t s)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_INV) default: return -1; }
}

int PK_SUFFIX(x_fwd_blocks)(int nx, int ny, int nz)
{
    switch (nx / 2) { PK_X_LENGTHS(PK_CASE_BLK) default: return -1; }
}

}  // namespace pk
