// k_ypass.hip -- transforms along y (steps 3 and 7 of the solve sequence in
// FluTAS Section 3.3.1), in place on the packed half spectrum S.
//
// On one GPU the whole grid is resident, so the x-to-y re-orientation of the
// paper's distributed code (its transposes 2 and 8) is replaced by a strided
// pass: a workgroup owns NB consecutive x-wavenumbers m of one z-plane k and
// transforms its NB columns S[k, :, m0:m0+NB] along y.  A wavefront's loads
// and stores are runs of NB contiguous complex values per y-row (128 B at the
// default tile), so the pass streams HBM once in and once out.
// The inverse is conj(FFT(conj)).
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

template <int N, bool INV, int V>
__global__ __launch_bounds__((YCfg<N, V>::NT)) void k_y(YArgs a0)
{
    if (gated_off(a0.batch, a0.gate, blockIdx.y)) return;
    YArgs a = a0;
    if (a.batch) a.S = a.batch[blockIdx.y].S;
    using C = YCfg<N, V>;
    constexpr int NB = C::NB, NT = C::NT;
    using Tile = LdsTile<R, N, NB, true, C::PAD>;
    __shared__ Cx<R> s_tile[Tile::elems];
    __shared__ Cx<R> s_tw[N];

    const int ntile = (a.M + NB - 1) / NB;
    const int bid = block_order(blockIdx.x, gridDim.x, a.reverse);
    const int tile_i = bid % ntile;
    const int k = bid / ntile;
    const int m0 = tile_i * NB;
    load_table(s_tw, (const Cx<R> *)a.tw, N);
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
    fft_tile<R, N, NB, NT, true, C::PAD, false, C::PV>(s_tw, 1, gload, gstore, tile);
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

}  // namespace PK_NS
using namespace PK_NS;

#define PK_CASE_Y(N) case N: return run_y<N>(a, s);

int PK_SUFFIX(launch_y)(const YArgs &a, hipStream_t s)
{
    switch (a.ny) { PK_LENGTHS(PK_CASE_Y) default: return -1; }
}

}  // namespace pk
