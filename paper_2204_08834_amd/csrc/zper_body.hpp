// zper_body.hpp -- the workgroup body of the periodic z pass (FFT along z,
// eigenvalue division, inverse FFT; see k_zperiodic.hip), shared by the
// per-group kernel and the work-list kernel.  Included inside namespace
// pk::PK_NS of a precision-templated source (R = PK_REAL).
#pragma once

template <int N> struct ZPCfg {
    static constexpr int NB0 = sizeof(R) == 4 ? 16 : 8;
    static constexpr int MAXE = sizeof(R) == 4 ? 16384 : 8192;
    static constexpr int NB1 = (NB0 * N <= MAXE) ? NB0 : ((MAXE / N) < 2 ? 2 : MAXE / N);
    static constexpr int NB = NB1 & ~1;  // even: the m = 0 role works on column pairs
    // 8 elements per thread (one radix-8 butterfly per pass): more waves in
    // flight for the small problems of a batch, and for long columns (FP32,
    // 256^3: 43 -> 39 us per pass with 512 threads instead of 256); FP32
    // columns of 96-192 points take 16 each
    static constexpr int NT = pick_nt(NB * N, (sizeof(R) == 4 && N > 64 && N < 256) ? 16 : 8);
    static constexpr int PAD = (NB >= 8) ? 1 : 0;
};

// One workgroup's work (block vb.x of problem vb.y); LDS carved from `lds`.
template <int N> struct ZPBody {
    using Cf = ZPCfg<N>;
    using Tile = LdsTile<R, N, Cf::NB, true, Cf::PAD>;
    static constexpr size_t TILE_B = sizeof(Cx<R>) * Tile::elems;
    static constexpr size_t LDS_BYTES = TILE_B + sizeof(Cx<R>) * N;

    static __device__ __forceinline__ void run(const ZArgs &a0, VBlock vb, int nspecial, char *lds)
    {
        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        ZArgs a = a0;
        if (a.batch) {
            const ProbPtrs &pq = a.batch[vb.y];
            a.S = pq.S;
            if (a.zero_mean_out) a.zero_mean_out = pq.scal;
        }
        constexpr int NB = Cf::NB, NT = Cf::NT;
        Cx<R> *s_tile = (Cx<R> *)lds;
        Cx<R> *s_tw = (Cx<R> *)(lds + TILE_B);
        load_table(s_tw, (const Cx<R> *)a.tw, N, NT);
        __syncthreads();

        const int M = a.M, ny = a.ny;
        const int ncol = ny * M;
        const size_t plane = (size_t)ncol;
        PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
        Tile tile{s_tile};
        auto lstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };

        if (vb.x >= nspecial) {
            const int q0 =
                block_order(vb.x - nspecial, vb.gx - nspecial, a.reverse) * NB;
            auto gload = [&](int b, int n) -> Cx<R> {
                const int q = q0 + b;
                if (q >= ncol) return {R(0), R(0)};
                return S[(size_t)n * plane + q];
            };
            fft_tile<R, N, NB, NT, true, Cf::PAD, false>(s_tw, 1, gload, lstore, tile);
            __syncthreads();
            auto gload2 = [&](int b, int n) -> Cx<R> {
                const int q = q0 + b;
                const int m = q % M, ky = q / M;
                if (q >= ncol || m == 0) return {R(0), R(0)};
                const double lam = a.lamx[m] + a.lamy[ky] + a.lamz[n];
                const R sc = R(a.inv_ntot / lam);
                return cconj(cscale(tile.at(b, n), sc));
            };
            auto gstore2 = [&](int b, int n, Cx<R> v) {
                const int q = q0 + b;
                if (q >= ncol || (q % M) == 0) return;
                S[(size_t)n * plane + q] = cconj(v);
            };
            fft_tile<R, N, NB, NT, true, Cf::PAD, true>(s_tw, 1, gload2, gstore2, tile);
            return;
        }

        // walls along x: every column m holds the real x-modes (2m, 2m+1) as
        // A + iB and takes the paths below (workgroups along m, coalesced);
        // otherwise only m = 0 (DC and Nyquist) does
        const int mblocks_y = a.xwall ? (M + NB - 1) / NB : 1;
        auto lamA_of = [&](int m) { return a.xwall ? a.lamx[2 * m] : a.lamx[0]; };
        auto lamB_of = [&](int m) { return a.xwall ? a.lamx[2 * m + 1] : a.lamx[M]; };
        if (a.ywall) {
            // ---- walls along y: each column (m, ky) holds A + iB (real modes
            // along y), which separate through the symmetry kz <-> -kz of the
            // same column.  A workgroup takes NB columns: NB values of ky at m = 0,
            // or NB consecutive m at one ky (walls along x)
            const int bx = vb.x;
            const int kyb = a.xwall ? bx / mblocks_y : bx * NB;
            const int mb = a.xwall ? (bx % mblocks_y) * NB : 0;
            auto colm = [&](int b) { return a.xwall ? mb + b : 0; };
            auto colky = [&](int b) { return a.xwall ? kyb : kyb + b; };
            auto inside = [&](int b) { return colky(b) < ny && colm(b) < M; };
            auto gload = [&](int b, int n) -> Cx<R> {
                if (!inside(b)) return {R(0), R(0)};
                return S[(size_t)n * plane + (size_t)colky(b) * M + colm(b)];
            };
            fft_tile<R, N, NB, NT, true, Cf::PAD, false>(s_tw, 1, gload, lstore, tile);
            __syncthreads();
            constexpr int NE = NB * N;
            constexpr int PER = (NE + NT - 1) / NT;
            Cx<R> o[PER];
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int u = threadIdx.x + e * NT;
                if (u >= NE) continue;
                const int b = u % NB, kz = u / NB;
                const int ky = colky(b), m = colm(b);
                if (!inside(b)) {
                    o[e] = {R(0), R(0)};
                    continue;
                }
                const int kzn = (N - kz) % N;
                const double ly = a.lamy[ky], lz = a.lamz[kz];
                const double lamA = lamA_of(m) + ly + lz, lamB = lamB_of(m) + ly + lz;
                const bool zero = m == 0 && ky == 0 && kz == 0 && !a.regular;
                const R sA = zero ? R(0) : R(a.inv_ntot / lamA);
                const R sB = R(a.inv_ntot / lamB);
                const Cx<R> z1 = tile.at(b, kz), z2 = cconj(tile.at(b, kzn));
                if (zero && a.zero_mean_out) *a.zero_mean_out = double(z1.re) * a.inv_ntot;
                const Cx<R> A = cscale(cadd(z1, z2), R(0.5) * sA);
                const Cx<R> B = cscale(cmul_mi(csub(z1, z2)), R(0.5) * sB);
                o[e] = cadd(A, cmul_pi(B));
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < PER; ++e) {
                const int u = threadIdx.x + e * NT;
                if (u < NE) tile.at(u % NB, u / NB) = o[e];
            }
            __syncthreads();
            auto gload3 = [&](int b, int n) -> Cx<R> { return cconj(tile.at(b, n)); };
            auto gstore3 = [&](int b, int n, Cx<R> v) {
                if (!inside(b)) return;
                S[(size_t)n * plane + (size_t)colky(b) * M + colm(b)] = cconj(v);
            };
            fft_tile<R, N, NB, NT, true, Cf::PAD, true>(s_tw, 1, gload3, gstore3, tile);
            return;
        }

        // ---- m = 0 column pairs ------------------------------------------------
        // A workgroup takes NP column pairs (ky, -ky): NP values of ky at m = 0,
        // or NP consecutive m at one ky (walls along x)
        constexpr int NP = NB / 2;
        const int mblocks_p = a.xwall ? (M + NP - 1) / NP : 1;
        const int bx = vb.x;
        const int kyp = a.xwall ? bx / mblocks_p : bx * NP;
        const int mp = a.xwall ? (bx % mblocks_p) * NP : 0;
        auto pm = [&](int i) { return a.xwall ? mp + i : 0; };
        auto pky = [&](int i) { return a.xwall ? kyp : kyp + i; };
        auto col_of = [&](int b, bool &valid, bool &dup) -> size_t {
            const int i = b / 2;
            const int ky = pky(i);
            valid = ky <= ny / 2 && pm(i) < M;
            const int kyv = valid ? ky : 0;
            const int kyn = (ny - kyv) % ny;
            dup = (b & 1) && (kyn == kyv);
            return (size_t)((b & 1) ? kyn : kyv) * M + (valid ? pm(i) : 0);
        };
        auto gload = [&](int b, int n) -> Cx<R> {
            bool valid, dup;
            const size_t col = col_of(b, valid, dup);
            if (!valid) return {R(0), R(0)};
            return S[(size_t)n * plane + col];
        };
        fft_tile<R, N, NB, NT, true, Cf::PAD, false>(s_tw, 1, gload, lstore, tile);
        __syncthreads();

        constexpr int NE = NP * N;
        constexpr int PER = (NE + NT - 1) / NT;
        Cx<R> o1[PER], o2[PER];
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int u = threadIdx.x + e * NT;
            if (u >= NE) continue;
            const int i = u % NP, kz = u / NP;
            const int kzn = (N - kz) % N;
            const int ky = pky(i), m = pm(i);
            if (ky > ny / 2 || m >= M) {
                o1[e] = o2[e] = {R(0), R(0)};
                continue;
            }
            const double lz = a.lamz[kz], ly = a.lamy[ky];
            const double lamA = lamA_of(m) + ly + lz, lamB = lamB_of(m) + ly + lz;
            const bool zero = m == 0 && ky == 0 && kz == 0 && !a.regular;
            const R sA = zero ? R(0) : R(a.inv_ntot / lamA);
            const R sB = R(a.inv_ntot / lamB);
            // (ky, kz)
            const Cx<R> z1 = tile.at(2 * i, kz), z2 = cconj(tile.at(2 * i + 1, kzn));
            if (zero && a.zero_mean_out)
                *a.zero_mean_out = double(z1.re) * a.inv_ntot;  // sum of f over the grid
            const Cx<R> A = cscale(cadd(z1, z2), R(0.5) * sA);
            const Cx<R> B = cscale(cmul_mi(csub(z1, z2)), R(0.5) * sB);
            o1[e] = cadd(A, cmul_pi(B));
            // (ky, -kz), recombined into column -ky at kz
            const Cx<R> w1 = tile.at(2 * i, kzn), w2 = cconj(tile.at(2 * i + 1, kz));
            const Cx<R> Am = cscale(cadd(w1, w2), R(0.5) * sA);
            const Cx<R> Bm = cscale(cmul_mi(csub(w1, w2)), R(0.5) * sB);
            o2[e] = cadd(cconj(Am), cmul_pi(cconj(Bm)));
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int u = threadIdx.x + e * NT;
            if (u >= NE) continue;
            const int i = u % NP, kz = u / NP;
            tile.at(2 * i, kz) = o1[e];
            tile.at(2 * i + 1, kz) = o2[e];
        }
        __syncthreads();
        auto gload3 = [&](int b, int n) -> Cx<R> { return cconj(tile.at(b, n)); };
        auto gstore3 = [&](int b, int n, Cx<R> v) {
            bool valid, dup;
            const size_t col = col_of(b, valid, dup);
            if (!valid || dup) return;
            S[(size_t)n * plane + col] = cconj(v);
        };
        fft_tile<R, N, NB, NT, true, Cf::PAD, true>(s_tw, 1, gload3, gstore3, tile);
    }
};

