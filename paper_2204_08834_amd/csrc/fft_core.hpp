// fft_core.hpp -- workgroup-level mixed-radix FFT engine for gfx950.
//
// The Fourier expansions of FluTAS Section 3.3.1 along x, y (and z when
// periodic) are computed as unnormalised forward DFTs
//     X[k] = sum_n x[n] exp(-2 pi i k n / N)
// of NB independent lines held by one workgroup.  The transform is a
// Stockham autosort sequence of radix-8/4/3/2 passes:
//   pass with radix R after sub-transforms of length Ns:
//     butterfly j in [0, N/R) reads x[j + r N/R], r = 0..R-1,
//     multiplies input r by w_{Ns R}^{r (j mod Ns)}, does an R-point DFT in
//     registers, and writes output r to ((j - j mod Ns) R + j mod Ns + r Ns).
// Pass 0 reads straight from global memory through a caller functor and the
// last pass writes through another, so one HBM read and one HBM write per
// element suffice; intermediate passes exchange through LDS.  Inverse
// transforms are done by the caller as conj(FFT(conj(x))).
//
// Lines are either "lines-fast" (consecutive lanes take consecutive lines --
// used for the strided y/z passes so that a wavefront's loads cover
// contiguous runs of the x-wavenumber) or "index-fast" (consecutive lanes take
// consecutive points of one line -- used for the contiguous x pass).
#pragma once
#include "common.hpp"

namespace pk {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ Cx<R> cconj(Cx<R> a) { return {a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return {a.re * s, a.im * s}; }
// multiply by -i
template <typename R>
__device__ __forceinline__ Cx<R> cmul_mi(Cx<R> a) { return {a.im, -a.re}; }
// multiply by +i
template <typename R>
__device__ __forceinline__ Cx<R> cmul_pi(Cx<R> a) { return {-a.im, a.re}; }

template <typename R> struct Const;
template <> struct Const<float> {
    static constexpr float rsqrt2 = 0.70710678118654752440f;
    static constexpr float sqrt3_2 = 0.86602540378443864676f;
};
template <> struct Const<double> {
    static constexpr double rsqrt2 = 0.70710678118654752440;
    static constexpr double sqrt3_2 = 0.86602540378443864676;
};

// ---------------------------------------------------------------------------
// radix plan: N = 2^a 3^b as radix-8 passes, then 4s, a 2, then 3s
// ---------------------------------------------------------------------------
struct RPlan {
    int count;
    int r[16];
};

constexpr RPlan make_rplan(int n)
{
    RPlan p{0, {0}};
    int a = 0, b = 0;
    while (n > 1 && n % 2 == 0) { n /= 2; ++a; }
    while (n > 1 && n % 3 == 0) { n /= 3; ++b; }
    int n8 = a / 3, n4 = 0, n2 = 0;
    if (a % 3 == 2) {
        n4 = 1;
    } else if (a % 3 == 1) {
        if (n8 > 0) { n8 -= 1; n4 = 2; } else { n2 = 1; }
    }
    for (int i = 0; i < n8; ++i) p.r[p.count++] = 8;
    for (int i = 0; i < n4; ++i) p.r[p.count++] = 4;
    for (int i = 0; i < n2; ++i) p.r[p.count++] = 2;
    for (int i = 0; i < b; ++i) p.r[p.count++] = 3;
    return p;
}

// plan variant: 0 = the order above, 1 = the same radices in reverse order
// (small radix first)
constexpr RPlan get_rplan(int n, int variant)
{
    RPlan p = make_rplan(n);
    if (variant == 1) {
        for (int i = 0; i < p.count / 2; ++i) {
            const int t = p.r[i];
            p.r[i] = p.r[p.count - 1 - i];
            p.r[p.count - 1 - i] = t;
        }
    }
    return p;
}

constexpr int rplan_ns(RPlan p, int pass)
{
    int ns = 1;
    for (int i = 0; i < pass; ++i) ns *= p.r[i];
    return ns;
}

// threads for a tile of `elems` complex values at `ept` values per thread,
// rounded to whole wavefronts, within [64, 1024]
constexpr int pick_nt(int elems, int ept)
{
    int nt = elems / ept;
    nt = (nt + 63) / 64 * 64;
    return nt < 64 ? 64 : (nt > 1024 ? 1024 : nt);
}

constexpr bool is_2a3b(int n)
{
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// ---------------------------------------------------------------------------
// R-point forward DFT butterflies in registers
// ---------------------------------------------------------------------------
template <typename R, int RAD> struct Bfly;

template <typename R> struct Bfly<R, 2> {
    static __device__ __forceinline__ void run(Cx<R> *x)
    {
        Cx<R> a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <typename R> struct Bfly<R, 3> {
    static __device__ __forceinline__ void run(Cx<R> *x)
    {
        const R s = Const<R>::sqrt3_2;
        Cx<R> sum = cadd(x[1], x[2]);
        Cx<R> a = {x[0].re - R(0.5) * sum.re, x[0].im - R(0.5) * sum.im};
        Cx<R> b = cscale(csub(x[1], x[2]), s);
        x[0] = cadd(x[0], sum);
        x[1] = cadd(a, cmul_mi(b));
        x[2] = cadd(a, cmul_pi(b));
    }
};

template <typename R> struct Bfly<R, 4> {
    static __device__ __forceinline__ void run(Cx<R> *x)
    {
        Cx<R> t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
        Cx<R> t2 = cadd(x[1], x[3]), t3 = cmul_mi(csub(x[1], x[3]));
        x[0] = cadd(t0, t2);
        x[2] = csub(t0, t2);
        x[1] = cadd(t1, t3);
        x[3] = csub(t1, t3);
    }
};

template <typename R> struct Bfly<R, 8> {
    static __device__ __forceinline__ void run(Cx<R> *x)
    {
        const R c = Const<R>::rsqrt2;
        Cx<R> e[4] = {x[0], x[2], x[4], x[6]};
        Cx<R> o[4] = {x[1], x[3], x[5], x[7]};
        Bfly<R, 4>::run(e);
        Bfly<R, 4>::run(o);
        // o[k] *= w8^k, w8 = exp(-i pi/4)
        o[1] = {c * (o[1].re + o[1].im), c * (o[1].im - o[1].re)};
        o[2] = cmul_mi(o[2]);
        o[3] = {c * (o[3].im - o[3].re), -c * (o[3].re + o[3].im)};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] = cadd(e[k], o[k]);
            x[k + 4] = csub(e[k], o[k]);
        }
    }
};

// ---------------------------------------------------------------------------
// LDS tile accessor
// ---------------------------------------------------------------------------
template <typename R, int N, int NB, bool LF, int PAD>
struct LdsTile {
    static constexpr int elems = LF ? N * (NB + PAD) : NB * (N + PAD);
    Cx<R> *base;
    __device__ __forceinline__ Cx<R> &at(int b, int n) const
    {
        return LF ? base[n * (NB + PAD) + b] : base[b * (N + PAD) + n];
    }
};

// ---------------------------------------------------------------------------
// one Stockham pass
// ---------------------------------------------------------------------------
template <typename R, int N, int NB, int NT, bool LF, int RAD, int NS, bool MIDSYNC,
          class Ld, class St>
__device__ __forceinline__ void stockham_pass(const Cx<R> *__restrict__ tw, int tws, Ld &ld,
                                              St &st)
{
    constexpr int NJ = N / RAD;
    constexpr int NBF = NB * NJ;
    constexpr int PER = (NBF + NT - 1) / NT;
    constexpr bool EXACT = (NBF % NT) == 0;
    Cx<R> v[PER][RAD];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int u = t + q * NT;
        if (EXACT || u < NBF) {
            const int b = LF ? (u % NB) : (u / NJ);
            const int j = LF ? (u / NB) : (u % NJ);
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[q][r] = ld(b, j + r * NJ);
        }
    }
    if (MIDSYNC) __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int u = t + q * NT;
        if (EXACT || u < NBF) {
            const int b = LF ? (u % NB) : (u / NJ);
            const int j = LF ? (u / NB) : (u % NJ);
            const int k = (NS == 1) ? 0 : (j % NS);
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r)
                    v[q][r] = cmul(v[q][r], tw[(r * k * (N / (NS * RAD))) * tws]);
            }
            Bfly<R, RAD>::run(v[q]);
            const int base = (j - k) * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r) st(b, base + r * NS, v[q][r]);
        }
    }
}

// ---------------------------------------------------------------------------
// full transform of a tile: gload -> passes -> gstore
//   gload(b, n) -> Cx<R>       : input element n of line b (pass 0)
//   gstore(b, n, Cx<R>)        : output element n of line b (last pass)
//   tile                       : LDS exchange buffer
// On return all threads have finished their stores (no trailing barrier).
// N == 1 is the identity.
// ---------------------------------------------------------------------------
template <typename R, int N, int NB, int NT, bool LF, int PAD, bool GL_LDS, int PASS, int END,
          int PV, class GL, class GS>
__device__ __forceinline__ void fft_passes(const Cx<R> *__restrict__ tw, int tws, GL &gload,
                                           GS &gstore, LdsTile<R, N, NB, LF, PAD> tile)
{
    // passes PASS .. END-1 of plan variant PV; pass 0 reads through gload,
    // pass END-1 writes through gstore, the others exchange through the LDS tile
    constexpr RPlan pl = get_rplan(N, PV);
    constexpr int RAD = pl.r[PASS];
    constexpr int NS = rplan_ns(pl, PASS);
    constexpr bool FIRST = PASS == 0;
    constexpr bool LAST = PASS == END - 1;
    auto lload = [&](int b, int n) { return tile.at(b, n); };
    auto lstore = [&](int b, int n, Cx<R> v) { tile.at(b, n) = v; };
    if constexpr (FIRST && LAST) {
        stockham_pass<R, N, NB, NT, LF, RAD, NS, true>(tw, tws, gload, gstore);
    } else if constexpr (FIRST) {
        stockham_pass<R, N, NB, NT, LF, RAD, NS, GL_LDS>(tw, tws, gload, lstore);
        __syncthreads();
    } else if constexpr (LAST) {
        stockham_pass<R, N, NB, NT, LF, RAD, NS, true>(tw, tws, lload, gstore);
    } else {
        stockham_pass<R, N, NB, NT, LF, RAD, NS, true>(tw, tws, lload, lstore);
        __syncthreads();
    }
    if constexpr (!LAST)
        fft_passes<R, N, NB, NT, LF, PAD, GL_LDS, PASS + 1, END, PV>(tw, tws, gload, gstore,
                                                                    tile);
}

// Inputs of pass 0 held in registers, so that a workgroup can load the next
// tile's inputs (prefetch) while it transforms the current one:
//   load(gload)  : v <- inputs of this thread's pass-0 butterflies
//   store(tile)  : pass-0 butterflies (no twiddles) -> LDS tile
// after which fft_passes continues from pass 1.
template <typename R, int N, int NB, int NT, bool LF, int PAD, int PV>
struct Pass0Regs {
    static constexpr RPlan pl = get_rplan(N, PV);
    static constexpr int RAD = pl.r[0], NJ = N / RAD, NBF = NB * NJ;
    static constexpr int PER = (NBF + NT - 1) / NT;
    static constexpr bool EXACT = (NBF % NT) == 0;
    Cx<R> v[PER][RAD];

    template <class GL>
    __device__ __forceinline__ void load(GL &gload)
    {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int u = threadIdx.x + q * NT;
            if (EXACT || u < NBF) {
                const int b = LF ? (u % NB) : (u / NJ);
                const int j = LF ? (u / NB) : (u % NJ);
#pragma unroll
                for (int r = 0; r < RAD; ++r) v[q][r] = gload(b, j + r * NJ);
            }
        }
    }
    __device__ __forceinline__ void store(LdsTile<R, N, NB, LF, PAD> tile)
    {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int u = threadIdx.x + q * NT;
            if (EXACT || u < NBF) {
                const int b = LF ? (u % NB) : (u / NJ);
                const int j = LF ? (u / NB) : (u % NJ);
                Bfly<R, RAD>::run(v[q]);
#pragma unroll
                for (int r = 0; r < RAD; ++r) tile.at(b, j * RAD + r) = v[q][r];
            }
        }
    }
};

// GL_LDS: gload reads the LDS tile itself (pass 0 then needs a barrier between
// its loads and its stores).
template <typename R, int N, int NB, int NT, bool LF, int PAD, bool GL_LDS, int PV = 0, class GL,
          class GS>
__device__ __forceinline__ void fft_tile(const Cx<R> *__restrict__ tw, int tws, GL &gload,
                                         GS &gstore, LdsTile<R, N, NB, LF, PAD> tile)
{
    if constexpr (N == 1) {
        constexpr int PER = (NB + NT - 1) / NT;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int b = threadIdx.x + q * NT;
            Cx<R> v;
            if (b < NB) v = gload(b, 0);
            __syncthreads();
            if (b < NB) gstore(b, 0, v);
        }
    } else {
        fft_passes<R, N, NB, NT, LF, PAD, GL_LDS, 0, make_rplan(N).count, PV>(tw, tws, gload,
                                                                              gstore, tile);
    }
}

// copy a global twiddle table (n entries) into LDS with the first nt threads
// (all of the workgroup by default); caller syncs
template <typename R>
__device__ __forceinline__ void load_table(Cx<R> *dst, const Cx<R> *__restrict__ src, int n,
                                           int nt = 0)
{
    const int step = nt > 0 ? nt : (int)blockDim.x;
    for (int t = threadIdx.x; t < n; t += step) dst[t] = src[t];
}

}  // namespace pk
