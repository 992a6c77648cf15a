// k_ypass.hip -- transforms along y (steps 3 and 7 of the solve sequence in
// FluTAS Section 3.3.1), in place on the packed half spectrum S.
//
// On one GPU the whole grid is resident, so the x-to-y re-orientation of the
// paper's distributed code (its transposes 2 and 8) is replaced by a strided
// pass: a workgroup owns NB consecutive x-wavenumbers m of one z-plane k and
// transforms its NB columns S[k, :, m0:m0+NB] along y.  A wavefront's loads
// and stores are runs of NB contiguous complex values per y-row (128 B at the
// default tile), so the pass streams HBM once in and once out.
// The inverse is conj(FFT(conj)).  With walls along y the columns are
// expanded in cosine or sine modes instead (k_yw below).
#include "fft_core.hpp"
#include "lengths.hpp"

#ifndef PK_REAL
#error "PK_REAL must be defined"
#endif

namespace pk {
namespace PK_NS {

using R = PK_REAL;

// Tile variants V (chosen per shape by the plan's autotuner):
//   bit 0: 256-byte row segments (twice the x-wavenumbers per workgroup)
//   bit 1: radix passes in reverse order (small radix first)
template <int N, int V> struct YCfg {
    // 128-byte row segments: 16 complex floats or 8 complex doubles; the
    // tile (up to 128 KB at N = 1024) stays in one workgroup's LDS
    static constexpr int NB0 = (sizeof(R) == 4 ? 16 : 8) * ((V & 1) ? 2 : 1);
    static constexpr int MAXE = sizeof(R) == 4 ? 16384 : 8192;
    static constexpr int NB = (NB0 * N <= MAXE) ? NB0 : ((MAXE / N) < 1 ? 1 : MAXE / N);
    static constexpr int NT = pick_nt(NB * N, sizeof(R) == 4 ? 16 : 8);
    static constexpr int PAD = (NB >= 8) ? 1 : 0;
    static constexpr int PV = (V & 2) ? 1 : 0;
};

// One workgroup's work: block vb.x (tile of NB x-wavenumbers of one plane)
// of problem vb.y; LDS carved from `lds` (LDS_BYTES).  Called by the
// per-group kernel and by the work-list kernel.
template <int N, bool INV, int V> struct YBody {
    using C = YCfg<N, V>;
    static constexpr int NB = C::NB, NT = C::NT;
    using Tile = LdsTile<R, N, NB, true, C::PAD>;
    static constexpr size_t TILE_B = sizeof(Cx<R>) * Tile::elems;
    static constexpr size_t LDS_BYTES = TILE_B + sizeof(Cx<R>) * N;

    static __device__ __forceinline__ void run(const YArgs &a0, VBlock vb, char *lds)
    {
        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        YArgs a = a0;
        if (a.batch) a.S = a.batch[vb.y].S;
        Cx<R> *s_tile = (Cx<R> *)lds;
        Cx<R> *s_tw = (Cx<R> *)(lds + TILE_B);

        const int ntile = (a.M + NB - 1) / NB;
        const int bid = block_order(vb.x, vb.gx, a.reverse);
        const int tile_i = bid % ntile;
        const int k = bid / ntile;
        const int m0 = tile_i * NB;
        load_table(s_tw, (const Cx<R> *)a.tw, N, NT);
        __syncthreads();

        Cx<R> *base = (Cx<R> *)a.S + (size_t)k * N * a.M + m0;
        const int M = a.M;
        auto gload = [&](int b, int n) -> Cx<R> {
            if (m0 + b >= M) return {R(0), R(0)};
            Cx<R> v = base[(size_t)n * M + b];
            return INV ? cconj(v) : v;
        };
        auto gstore = [&](int b, int n, Cx<R> v) {
            if (m0 + b >= M) return;
            base[(size_t)n * M + b] = INV ? cconj(v) : v;
        };
        Tile tile{s_tile};
        constexpr RPlan pl = get_rplan(N, C::PV);
        constexpr int R0 = pl.count >= 2 ? pl.r[0] : 1;
        // FP32 inverse: pass 0 gives each thread the butterfly pair
        // (p, NJ - p) (or (0, NJ/2)) instead of the plain mapping's
        // butterflies NT/NB apart (as the wall pass does, where the pair
        // shares its inputs).
        // Measured on MI355X at 512x512x256: inverse 105.6 -> 99.5 us; the
        // forward pass and FP64 ran 1-3 % slower with it.
        constexpr bool PAIR = INV && sizeof(R) == 4;
        if constexpr (PAIR && pl.count >= 2 && (N / R0) % 2 == 0) {
            constexpr int RAD = R0, NJ = N / RAD, U = NJ / 2, NU = NB * U;
            constexpr int PER = (NU + NT - 1) / NT;
            Cx<R> v1[PER][RAD], v2[PER][RAD];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u % NB, pp = u / NB;
                const int j1 = pp, j2 = pp == 0 ? NJ / 2 : NJ - pp;
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    v1[q][r] = gload(b, j1 + r * NJ);
                    v2[q][r] = gload(b, j2 + r * NJ);
                }
            }
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u % NB, pp = u / NB;
                const int j1 = pp, j2 = pp == 0 ? NJ / 2 : NJ - pp;
                Bfly<R, RAD>::run(v1[q]);
                Bfly<R, RAD>::run(v2[q]);
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    tile.at(b, j1 * RAD + r) = v1[q][r];
                    tile.at(b, j2 * RAD + r) = v2[q][r];
                }
            }
            __syncthreads();
            auto gnone = [&](int, int) -> Cx<R> { return {R(0), R(0)}; };
            fft_passes<R, N, NB, NT, true, C::PAD, false, 1, pl.count, C::PV>(s_tw, 1, gnone,
                                                                              gstore, tile);
        } else {
            fft_tile<R, N, NB, NT, true, C::PAD, false, C::PV>(s_tw, 1, gload, gstore, tile);
        }
    }
};

template <int N, bool INV, int V>
__global__ __launch_bounds__((YCfg<N, V>::NT)) void k_y(YArgs a0)
{
    using B = YBody<N, INV, V>;
    __shared__ __align__(16) char s_lds[B::LDS_BYTES];
    B::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, s_lds);
}

// ---------------------------------------------------------------------------
// Walls along y: expansion in the cosine (Neumann) or sine (Dirichlet) basis
// of the cell-centred operator, phi_k(j) = cos(pi k (j+1/2)/n) or
// sin(pi (k+1)(j+1/2)/n), computed with one n-point FFT per column
// (Makhoul's reordering, written for complex columns: every step is linear
// over the complex numbers, so the real and imaginary parts of a column are
// expanded independently, as the x-wavenumber columns require):
//   forward cosine:  v[j] = c[r(j)],  r(j) = 2j (2j < n) or 2n-1-2j,
//                    V = FFT(v),  C[k] = (w_k V[k] + conj(w_k) V[(n-k) mod n]) / 2,
//                    w_k = exp(-i pi k / (2n));
//   forward sine:    the cosine transform of (-1)^j c[j], read out reversed
//                    (S[k] = C'[n-1-k]);
//   inverse cosine:  W[k] = conj(w_k) (C[k] - i C[n-k]),  C[n] = 0 (formed as
//                    the FFT's first pass loads it),
//                    v = FFT^-1(W) (unnormalised),  c[r(j)] = v[j]  (times n,
//                    like the periodic pass: 1/ny is applied in the z step);
//   inverse sine:    the inverse cosine transform of C'[k] = S[n-1-k], times
//                    (-1)^j.
// Forward: the last Stockham pass takes butterfly pairs (p, NJ - p), so V[k]
// and V[n-k] meet in one thread and the coefficients are stored from
// registers (lengths whose last pass has an odd number of butterflies store
// the FFT back into the LDS tile and combine the pairs from there).  Inverse:
// W is formed as pass 0 loads it.  Row runs of 128 bytes as in the periodic
// pass, narrower only where the tile and the tables would not fit.
template <int N> struct YWCfg {
    static constexpr int NB0 = sizeof(R) == 4 ? 16 : 8;
    // one NB x N tile (plus padding) and the N-entry twiddle table within
    // ~150 KB of LDS
    static constexpr int ELEMS = 150 * 1024 / (int)sizeof(Cx<R>);
    static constexpr int NBMAX = ELEMS / N - 1;  // N (NB + PAD) + N <= ELEMS
    static constexpr int NB1 = NB0 < NBMAX ? NB0 : NBMAX;
    static constexpr int NB2 = NB1 >= 16 ? 16 : (NB1 >= 8 ? 8 : (NB1 >= 4 ? 4 : (NB1 >= 2 ? 2 : 1)));
    // the padding column of tiles with 8 or more lines must fit as well
    static constexpr int NB = (NB2 >= 8 && N * (NB2 + 2) > ELEMS) ? NB2 / 2 : NB2;
    static constexpr int NT = pick_nt(NB * N, sizeof(R) == 4 ? 16 : 8);
    // the exp(-i pi k/(2n)) table goes to LDS; the padding column of the tile
    // is dropped where that keeps a resident workgroup per CU
    static constexpr int LDS_CU = 160 * 1024;
    static constexpr int PAD0 = (NB >= 8) ? 1 : 0;
    static constexpr int B_PAD = (N * (NB + PAD0) + 2 * N) * (int)sizeof(Cx<R>);
    static constexpr int B_NOPAD = (N * NB + 2 * N) * (int)sizeof(Cx<R>);
    static constexpr int B_GLB = (N * (NB + PAD0) + N) * (int)sizeof(Cx<R>);
    static constexpr bool FITS_PAD = LDS_CU / B_PAD == LDS_CU / B_GLB;
    static constexpr bool FITS_NOPAD = LDS_CU / B_NOPAD == LDS_CU / B_GLB;
    static constexpr int PAD = FITS_PAD ? PAD0 : (FITS_NOPAD ? 0 : PAD0);
    static constexpr bool W4_LDS = FITS_PAD || FITS_NOPAD;
};

__device__ __forceinline__ int wall_reorder(int j, int n) { return 2 * j < n ? 2 * j : 2 * n - 1 - 2 * j; }

// WV (autotuned variant) of the forward pass: bit 0 takes the transform's
// last pass into the LDS tile and combines the coefficient pairs from there
// (as the lengths whose last pass has an odd number of butterflies do)
// instead of the fused pair pass (FP64 at 512x512x256: 210 against 227 us;
// FP32 alike).  SINE: Dirichlet walls (sine basis), a compile-time constant
// so that every row address is a fixed function of the butterfly index.
template <int N, bool INV, int WV, bool SINE>
__global__ __launch_bounds__((YWCfg<N>::NT)) void k_yw(YArgs a0)
{
    if (gated_off(a0.batch, a0.gate, blockIdx.y)) return;
    YArgs a = a0;
    if (a.batch) a.S = a.batch[blockIdx.y].S;
    using C = YWCfg<N>;
    constexpr int NB = C::NB, NT = C::NT;
    using Tile = LdsTile<R, N, NB, true, C::PAD>;
    __shared__ Cx<R> s_tile[Tile::elems];
    __shared__ Cx<R> s_tw[N];
    __shared__ Cx<R> s_w4l[C::W4_LDS ? N : 1];  // exp(-i pi k / (2n))

    constexpr bool sine = SINE;
    const int ntile = (a.M + NB - 1) / NB;
    const int bid = block_order(blockIdx.x, gridDim.x, a.reverse);
    const int tile_i = bid % ntile;
    const int k = bid / ntile;
    const int m0 = tile_i * NB;
    load_table(s_tw, (const Cx<R> *)a.tw, N);
    if constexpr (C::W4_LDS) {
        // the forward pass keeps w_k / 2 (exact: a power-of-two scaling)
        const Cx<R> *src = (const Cx<R> *)a.tw4;
        for (int t = threadIdx.x; t < N; t += NT)
            s_w4l[t] = INV ? src[t] : Cx<R>{src[t].re * R(0.5), src[t].im * R(0.5)};
    }
    __syncthreads();
    auto w4 = [&]() {
        if constexpr (C::W4_LDS)
            return (const Cx<R> *)s_w4l;
        else
            return gbl((const Cx<R> *)a.tw4);
    }();
    // w_k / 2 for the forward pass
    auto whalf = [&](int kk) -> Cx<R> {
        const Cx<R> w = w4[kk];
        if constexpr (C::W4_LDS) return w;
        return Cx<R>{w.re * R(0.5), w.im * R(0.5)};
    };

    const int M = a.M;
    PK_GLOBAL Cx<R> *base = gbl((Cx<R> *)a.S) + (size_t)k * N * M + m0;
    Tile tile{s_tile};
    if constexpr (!INV) {
        Tile out = tile;  // the last pass stores back into the tile
        auto gload = [&](int b, int n) -> Cx<R> {
            if (m0 + b >= M) return {R(0), R(0)};
            const int r = wall_reorder(n, N);
            const Cx<R> v = base[(size_t)r * M + b];
            return (sine && (r & 1)) ? Cx<R>{-v.re, -v.im} : Cx<R>{v.re, v.im};
        };
        auto lstore = [&](int b, int n, Cx<R> v) { out.at(b, n) = v; };
        constexpr RPlan pl = make_rplan(N);
        constexpr int LR = pl.count >= 2 ? pl.r[pl.count - 1] : 1;
        if constexpr (pl.count >= 2 && (N / LR) % 2 == 0 && (WV & 1) == 0) {
            // every pass but the last into LDS; the last pass with butterfly
            // pairs (p, NJ - p) (or (0, NJ/2)), so that V[k] and V[N-k] meet in
            // one thread and the coefficients are stored from registers:
            //   C[k] = (w_k V[k] + conj(w_k) V[N-k]) / 2, likewise C[N-k]
            fft_passes<R, N, NB, NT, true, C::PAD, false, 0, pl.count - 1, 0>(s_tw, 1, gload,
                                                                              lstore, tile);
            __syncthreads();
            constexpr int RAD = LR, NJ = N / LR, U = NJ / 2, NU = NB * U;
            constexpr int PER = (NU + NT - 1) / NT;
            auto emit = [&](int b, int kk, Cx<R> vk, Cx<R> vc) {
                // with S = V[k] + V[N-k], D = V[k] - V[N-k] and h = w/2:
                //   C[k]   = h_k S + i h_k^i D   = (h^r S^r - h^i D^i, h^r S^i + h^i D^r),
                //   C[N-k] = h_{N-k} S - i h^i D (the same S and D), where
                //   h_{N-k} = -i conj(h_k) = (-h^i, -h^r): one table entry
                const Cx<R> S = {vk.re + vc.re, vk.im + vc.im};
                const Cx<R> D = {vk.re - vc.re, vk.im - vc.im};
                const Cx<R> h = whalf(kk);
                put(base + (size_t)(sine ? N - 1 - kk : kk) * M + b,
                    Cx<R>{h.re * S.re - h.im * D.im, h.re * S.im + h.im * D.re});
                if (kk != 0 && 2 * kk != N)
                    put(base + (size_t)(sine ? kk - 1 : N - kk) * M + b,
                        Cx<R>{-(h.im * S.re + h.re * D.im), h.re * D.re - h.im * S.im});
            };
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u % NB, pp = u / NB;
                const int j1 = pp, j2 = pp == 0 ? NJ / 2 : NJ - pp;
                Cx<R> v1[RAD], v2[RAD];
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    v1[r] = out.at(b, j1 + r * NJ);
                    v2[r] = out.at(b, j2 + r * NJ);
                }
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    v1[r] = cmul(v1[r], s_tw[r * j1]);
                    v2[r] = cmul(v2[r], s_tw[r * j2]);
                }
                Bfly<R, RAD>::run(v1);
                Bfly<R, RAD>::run(v2);
                if (m0 + b >= M) continue;
                if (pp == 0) {
                    // butterfly 0: k = r NJ with partner (RAD - r) NJ; k = 0 alone
                    emit(b, 0, v1[0], v1[0]);
#pragma unroll
                    for (int r = 1; r < RAD; ++r)
                        if (r <= RAD - r) emit(b, r * NJ, v1[r], v1[RAD - r]);
                    // butterfly NJ/2: k = NJ/2 + r NJ with partner r <-> RAD-1-r
#pragma unroll
                    for (int r = 0; r < RAD; ++r)
                        if (r <= RAD - 1 - r) emit(b, NJ / 2 + r * NJ, v2[r], v2[RAD - 1 - r]);
                } else {
#pragma unroll
                    for (int r = 0; r < RAD; ++r) emit(b, j1 + r * NJ, v1[r], v2[RAD - 1 - r]);
                }
            }
        } else {
            fft_tile<R, N, NB, NT, true, C::PAD, false>(s_tw, 1, gload, lstore, tile);
            __syncthreads();
            for (int e = threadIdx.x; e < NB * N; e += NT) {
                const int b = e % NB, kk = e / NB;
                if (m0 + b >= M) continue;
                const Cx<R> h = whalf(kk);
                const Cx<R> v1 = out.at(b, kk), v2 = out.at(b, kk == 0 ? 0 : N - kk);
                const Cx<R> S = {v1.re + v2.re, v1.im + v2.im};
                const Cx<R> D = {v1.re - v2.re, v1.im - v2.im};
                put(base + (size_t)(sine ? N - 1 - kk : kk) * M + b,
                    Cx<R>{h.re * S.re - h.im * D.im, h.re * S.im + h.im * D.re});
            }
        }
    } else {
        // W[k] = conj(w_k) (C[k] - i C[n-k]) formed in pass 0's loads from the
        // coefficient rows k and n-k (C[n] = 0; read reversed for sines); the
        // inverse FFT as conj(FFT(conj)).  (Staging the rows in the tile
        // first, one read of each, measured slower on MI355X than reading
        // each row twice; pass 0 with butterfly pairs below reads each once
        // from registers.)
        auto coef = [&](int b, int kk) -> Cx<R> {
            if (kk >= N) return {R(0), R(0)};
            const Cx<R> g = base[(size_t)(sine ? N - 1 - kk : kk) * M + b];
            return {g.re, g.im};
        };
        auto gload = [&](int b, int n) -> Cx<R> {
            if (m0 + b >= M) return {R(0), R(0)};
            const Cx<R> c1 = coef(b, n), c2 = n == 0 ? Cx<R>{R(0), R(0)} : coef(b, N - n);
            return cconj(cmul(cconj(w4[n]), csub(c1, cmul_pi(c2))));
        };
        auto gstore = [&](int b, int n, Cx<R> v) {
            if (m0 + b >= M) return;
            const int r = wall_reorder(n, N);
            const R sg = (sine && (r & 1)) ? R(-1) : R(1);
            put(base + (size_t)r * M + b, Cx<R>{sg * v.re, -sg * v.im});
        };
        constexpr RPlan pl = make_rplan(N);
        constexpr int R0 = pl.count >= 2 ? pl.r[0] : 1;
        if constexpr (pl.count >= 2 && (N / R0) % 2 == 0) {
            // pass 0 with butterfly pairs (p, NJ - p) (or (0, NJ/2)): W[n] and
            // W[N-n] need the same two coefficient rows, so one thread reads
            // each pair once and forms both,
            //   W[n] = conj(w_n) (A - i B),  W[N-n] = i w_n (B - i A),
            //   A = C[n], B = C[N-n]  (w_{N-n} = -i conj(w_n)),
            // returned conjugated (the inverse runs as conj(FFT(conj))).
            constexpr int RAD = R0, NJ = N / RAD, U = NJ / 2, NU = NB * U;
            constexpr int PER = (NU + NT - 1) / NT;
            auto wpair = [&](int n, Cx<R> A, Cx<R> B, Cx<R> &wn, Cx<R> &wc) {
                const Cx<R> w = w4[n];
                wn = cconj(cmul(cconj(w), csub(A, cmul_pi(B))));
                wc = cconj(cmul_pi(cmul(w, csub(B, cmul_pi(A)))));
            };
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int u = threadIdx.x + q * NT;
                if (NU % NT != 0 && u >= NU) break;
                const int b = u % NB, pp = u / NB;
                const int j1 = pp, j2 = pp == 0 ? NJ / 2 : NJ - pp;
                const bool live = m0 + b < M;
                auto cf = [&](int kk) -> Cx<R> { return live ? coef(b, kk) : Cx<R>{R(0), R(0)}; };
                Cx<R> v1[RAD], v2[RAD];
                if (pp == 0) {
                    // butterfly 0: n = r NJ with partner (RAD - r) NJ (n = 0:
                    // C[N] = 0); butterfly NJ/2: n = NJ/2 + r NJ, partner
                    // r <-> RAD-1-r
                    Cx<R> dummy;
                    wpair(0, cf(0), Cx<R>{R(0), R(0)}, v1[0], dummy);
                    // (an index that is its own partner, n = N/2, takes wn)
#pragma unroll
                    for (int r = 1; r < RAD; ++r)
                        if (r <= RAD - r) {
                            const Cx<R> A = cf(r * NJ), B = cf(N - r * NJ);
                            wpair(r * NJ, A, B, v1[r], r == RAD - r ? dummy : v1[RAD - r]);
                        }
#pragma unroll
                    for (int r = 0; r < RAD; ++r)
                        if (r <= RAD - 1 - r) {
                            const int n = NJ / 2 + r * NJ;
                            const Cx<R> A = cf(n), B = cf(N - n);
                            wpair(n, A, B, v2[r], r == RAD - 1 - r ? dummy : v2[RAD - 1 - r]);
                        }
                } else {
#pragma unroll
                    for (int r = 0; r < RAD; ++r) {
                        const int n = j1 + r * NJ;
                        const Cx<R> A = cf(n), B = cf(N - n);
                        wpair(n, A, B, v1[r], v2[RAD - 1 - r]);
                    }
                }
                Bfly<R, RAD>::run(v1);
                Bfly<R, RAD>::run(v2);
#pragma unroll
                for (int r = 0; r < RAD; ++r) {
                    tile.at(b, j1 * RAD + r) = v1[r];
                    tile.at(b, j2 * RAD + r) = v2[r];
                }
            }
            __syncthreads();
            auto gnone = [&](int, int) -> Cx<R> { return {R(0), R(0)}; };
            fft_passes<R, N, NB, NT, true, C::PAD, false, 1, pl.count, 0>(s_tw, 1, gnone, gstore,
                                                                          tile);
        } else {
            fft_tile<R, N, NB, NT, true, C::PAD, false>(s_tw, 1, gload, gstore, tile);
        }
    }
}

template <int N> static int run_yw(const YArgs &a, hipStream_t s)
{
    using C = YWCfg<N>;
    const int ntile = (a.M + C::NB - 1) / C::NB;
    const dim3 grid(ntile * a.nz, a.batch ? a.nbatch : 1);
    const bool sn = a.bc == 2;
    if (a.inverse) {
        if (sn)
            hipLaunchKernelGGL((k_yw<N, true, 0, true>), grid, dim3(C::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_yw<N, true, 0, false>), grid, dim3(C::NT), 0, s, a);
    } else if (a.variant & 1) {
        if (sn)
            hipLaunchKernelGGL((k_yw<N, false, 1, true>), grid, dim3(C::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_yw<N, false, 1, false>), grid, dim3(C::NT), 0, s, a);
    } else {
        if (sn)
            hipLaunchKernelGGL((k_yw<N, false, 0, true>), grid, dim3(C::NT), 0, s, a);
        else
            hipLaunchKernelGGL((k_yw<N, false, 0, false>), grid, dim3(C::NT), 0, s, a);
    }
    return (int)hipGetLastError();
}

template <int N, int V> static int run_yv(const YArgs &a, hipStream_t s)
{
    using C = YCfg<N, V>;
    const int ntile = (a.M + C::NB - 1) / C::NB;
    const dim3 grid(ntile * a.nz, a.batch ? a.nbatch : 1);
    if (a.inverse)
        hipLaunchKernelGGL((k_y<N, true, V>), grid, dim3(C::NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_y<N, false, V>), grid, dim3(C::NT), 0, s, a);
    return (int)hipGetLastError();
}

// short transforms have a single tile shape worth having
template <int N> static int run_y(const YArgs &a, hipStream_t s)
{
    if (a.bc != 0) return run_yw<N>(a, s);
    if constexpr (N < 64) {
        return run_yv<N, 0>(a, s);
    } else {
        switch (a.variant & 3) {
        case 1: return run_yv<N, 1>(a, s);
        case 2: return run_yv<N, 2>(a, s);
        case 3: return run_yv<N, 3>(a, s);
        default: return run_yv<N, 0>(a, s);
        }
    }
}

// ---------------------------------------------------------------------------
// Work list: periodic y passes of problems of different shapes in one launch
// (class = the transform length, tile variant 0, at most YL_NT threads).
// ---------------------------------------------------------------------------
constexpr int YL_NT = 256;
#define PK_YL_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

template <bool INV>
__global__ __launch_bounds__(YL_NT) void k_y_list(ListArgs<YArgs>)
{
    extern __shared__ __align__(16) char s_dyn[];
    const PK_KARG ListArgs<YArgs> *L = list_args<YArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const YArgs arg = L->a[g];
    switch (L->cls[g]) {
#define PK_YL_CASE(N)                                                                  \
    case N:                                                                            \
        if constexpr (YCfg<N, 0>::NT <= YL_NT) YBody<N, INV, 0>::run(arg, vb, s_dyn); \
        break;
        PK_YL_LENGTHS(PK_YL_CASE)
#undef PK_YL_CASE
    default: break;
    }
}

// class info of a y record for the list kernel: false when it has none
static bool y_list_class(const YArgs &a, int &nt, int &gx, size_t &lds)
{
    if (a.bc != 0) return false;
    switch (a.ny) {
#define PK_YL_INFO(N)                                                   \
    case N: {                                                           \
        using B = YBody<N, false, 0>;                                   \
        if (B::NT > YL_NT) return false;                                \
        nt = B::NT;                                                     \
        gx = (a.M + B::NB - 1) / B::NB * a.nz;                          \
        lds = B::LDS_BYTES;                                             \
        return true;                                                    \
    }
        PK_YL_LENGTHS(PK_YL_INFO)
#undef PK_YL_INFO
    default: return false;
    }
}

}  // namespace PK_NS
using namespace PK_NS;

int PK_SUFFIX(launch_y)(const YArgs &a, hipStream_t s);

int PK_SUFFIX(launch_y_list)(const YArgs *a, int n, hipStream_t s)
{
    ListArgs<YArgs> L{};
    size_t lds = 0;
    int total = 0;
    const bool inv = n > 0 && a[0].inverse;
    auto flush = [&]() -> int {
        if (L.nseg == 0) return 0;
        L.start[L.nseg] = total;
        if (inv)
            hipLaunchKernelGGL(k_y_list<true>, dim3(total), dim3(YL_NT), lds, s, L);
        else
            hipLaunchKernelGGL(k_y_list<false>, dim3(total), dim3(YL_NT), lds, s, L);
        L.nseg = 0;
        total = 0;
        lds = 0;
        return (int)hipGetLastError();
    };
    for (int i = 0; i < n; ++i) {
        if ((a[i].inverse != 0) != inv) return (int)hipErrorInvalidValue;
        if (a[i].ny == 1) continue;  // the identity
        int nt = 0, gx = 0;
        size_t b = 0;
        if (!y_list_class(a[i], nt, gx, b)) {
            const int e = PK_SUFFIX(launch_y)(a[i], s);
            if (e) return e;
            continue;
        }
        const int g = L.nseg++;
        L.start[g] = total;
        L.gx[g] = gx;
        L.cls[g] = a[i].ny;
        L.nt[g] = nt;
        L.a[g] = a[i];
        total += gx * (a[i].batch ? a[i].nbatch : 1);
        lds = lds > b ? lds : b;
        if (L.nseg == LIST_MAX_SEG) {
            const int e = flush();
            if (e) return e;
        }
    }
    return flush();
}

#define PK_CASE_Y(N) case N: return run_y<N>(a, s);

int PK_SUFFIX(launch_y)(const YArgs &a, hipStream_t s)
{
    switch (a.ny) { PK_LENGTHS(PK_CASE_Y) default: return -1; }
}

}  // namespace pk
