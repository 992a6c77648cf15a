// k_zwalls.hip -- z solve for wall-bounded boxes (steps 4-6 of the solve
// sequence in FluTAS Section 3.3.1: the tridiagonal system along z of each
// wavenumber pair, solved by Gauss elimination).
//
// For wavenumbers (m, ky) the transformed equation along z is, per row k,
//     a p[k-1] + (lam - 2a) p[k] + a p[k+1] = fhat[k] / (nx ny),  a = 1/dz^2,
// lam = lam_x(m) + lam_y(ky), lam(j) = -(4/h^2) sin^2(pi j/n); the mirrored
// ghost at the walls turns the end rows into (lam - a) on the diagonal; with
// zero-value (Dirichlet) walls the ghost is the negated wall cell and the end
// rows get (lam - 3a).
// Divided by a: p[k-1] + beta_k p[k] + p[k+1] = d[k], beta_k = sigma - 2
// (sigma = lam dz^2), sigma - 1 on the end rows (sigma alone when nz = 1);
// Dirichlet: sigma - 3 on the end rows (sigma - 4 when nz = 1).
//
// Gauss elimination without pivoting (Thomas):
//     c'_k = 1/(beta_k - c'_{k-1}),  d'_k = (d_k - d'_{k-1}) c'_k,
//     p_k  = d'_k - c'_k p_{k+1}.
// Deficit form.  For the lowest wavenumbers sigma is tiny (about -1.5e-4 for
// (m, ky) = (1, 0) on 512x512x256), and forming beta = sigma - 2 rounds away
// most of sigma (a 1e-12 relative error in FP64, 3e-3 in FP32).  With
// s = -sigma >= 0, u_k = -c'_k and v_k = 1 - u_k, every pivot is a sum of
// non-negative terms:
//     |pivot_0| = 1 + s,  |pivot_k| = 1 + s + v_{k-1},  |pivot_{nz-1}| = s + v_{nz-2},
//     u_k = 1/|pivot_k|,  v_k = (|pivot_k| - 1) u_k,
//     d'_k = (d'_{k-1} - d_k) u_k,  p_k = d'_k + p_{k+1} - v_k p_{k+1},
// so s keeps its full relative precision and the near-singular last pivot is
// formed without cancellation.  Dirichlet walls add 2 to the first and the
// last pivot (|pivot_0| = 3 + s, |pivot_{nz-1}| = 2 + s + v_{nz-2}): the
// system is then regular for every wavenumber, (0, 0) included.
//
// Partitioned form: a column is spread over C threads, each holding a chunk of
// L rows in registers; HBM is read and written once.  Every recurrence is
// composed per chunk and then across chunks through LDS:
//   1. v is a Moebius map of v_{k-1}: v -> (s + v)/(1 + s + v), matrix
//      [[1, s], [1, 1+s]]/(1+s) (all entries >= 0, so products do not cancel;
//      row 0 maps anything to s/(1+s)).  The product of the preceding chunks
//      gives v entering the chunk.
//   2. d' is affine in the value entering the chunk: d'_k = D_k + G_k d'_{s-1}.
//   3. p is affine in the value leaving the chunk: p_k = X_k + H_k p_{e+1}.
// Each composition is a short sequential scan over the C chunks.
//
// Column m = 0 of the packed spectrum holds two real x-modes (DC and
// Nyquist) combined as A + iB; after the y transform they separate as
//     A(ky) = (Z(ky) + conj Z(-ky))/2,  B(ky) = (Z(ky) - conj Z(-ky))/(2i).
// The first `nspecial` workgroups take these virtual columns (pairs ky,
// -ky) and recombine the results with a lane exchange.  With walls along y
// the y coefficients are real-linear: column (0, ky) holds A + iB itself, and
// the lanes of a pair take its real and imaginary parts.  With walls along x
// every column m holds two real x-modes (2m, 2m+1) as A + iB, so every column
// takes this path (eigenvalues lam_x(2m), lam_x(2m+1)).  The singular column
// (m, ky) = (0, 0) -- the zero wavenumber -- is solved in FP64 whatever the
// precision: its right-hand side mean is removed (this removes mean(f), which
// is reported), p is pinned by the zero-mean gauge, and the Neumann problem
// p[k-1] - 2p[k] + p[k+1] = g[k] is integrated twice (face fluxes are the
// running sums of g, p the running sums of the fluxes), then made zero-mean.
#include "fft_core.hpp"
#include "lengths.hpp"

#ifndef PK_REAL
#error "PK_REAL must be defined"
#endif

namespace pk {
namespace PK_NS {

using R = PK_REAL;

// 1/x from the hardware reciprocal refined by Newton steps r += r (1 - x r)
// (one for FP32, two for FP64): within an ulp, far shorter than the IEEE
// division sequence on the dependent elimination chain.  x > 0 and normal.
__device__ __forceinline__ float rcp_nr(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, r, 1.0f), r, r);
}
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    return fma(fma(-x, r, 1.0), r, r);
}

// Index of field f of the LDS slot of chunk cc, lane w (C chunks of W
// lanes): the fields of a slot are grouped by P, and group g of every
// (chunk, lane) is stored lane-contiguous, so that a wavefront reading or
// writing one group of its lanes' slots touches consecutive words (no LDS
// bank conflicts).  P = 1 stores every field lane-contiguous; P = 4 with
// FP32 gives one 16-byte access per lane and group.  A slot of consecutive
// reals per lane (the layout before) put the lanes of the FP64 and real
// solves 32-64 bytes apart: bank conflicts took most of their cycles.
// Measured at 512x512x256: P = 4 for complex FP32 columns (94 against 101
// us), P = 1 for FP64 and for the real systems (FP32 113 against 139 us).
template <int P>
__device__ __forceinline__ size_t zw_slot(int f, int cc, int w, int C, int W)
{
    return (((size_t)(f / P) * C + cc) * W + w) * P + (f % P);
}

// One workgroup's work (block vb.x of problem vb.y): C chunks of L rows of W
// columns; `smem_d` holds the dynamic LDS of zw_lds_bytes().
template <int L, int W, bool STR = false> struct ZWBody {
    static __device__ __forceinline__ void run(const ZArgs &a0, VBlock vb, int C, int nspecial,
                                               double *smem_d)
    {
        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        ZArgs a = a0;
        if (a.batch) {
            const ProbPtrs &pq = a.batch[vb.y];
            a.S = pq.S;
            if (a.zero_mean_out) a.zero_mean_out = pq.scal;
        }
        // C*W slots of 4 reals in lane-contiguous groups (zw_slot)
        R *buf = (R *)smem_d;
        double *zbuf = smem_d + ((C * W * 4 * sizeof(R) + 7) / 8);  // 3*C doubles

        const int t = threadIdx.x;
        const int w = t % W, c = t / W;
        constexpr int P = sizeof(R) == 4 ? 4 : 1;
        auto sl = [&](int f, int cc) -> R & { return buf[zw_slot<P>(f, cc, w, C, W)]; };
        const int nz = a.nz, M = a.M, ny = a.ny;
        const size_t plane = (size_t)ny * M;
        PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
        const int s = c * L;
        const int e = (s + L < nz) ? s + L : nz;  // chunk rows [s, e)
        const bool special = vb.x < nspecial;
        const double scale = a.dz2 * a.inv_nxny;
        // stretched z: the rows' coefficients from the table (ZArgs::zrow); s of
        // the column is -(lam_x + lam_y) times dz^2 (uniform rows, divided by
        // 1/dz^2) or, per row, times h_k (stretched rows, multiplied by h_k)
        const double *zrow = a.zrow;
        auto zr = [&](int k, int f) -> double { return zrow[8 * k + f]; };
        const double sfac = STR ? 1.0 : a.dz2;
        // stretched rows in FP32: a, c, h and D of every row (padding rows
        // included) staged in LDS, since the recurrences read them on their
        // dependency chains (FP32 z pass at 512x512x256: 141 against 190 us;
        // FP64 keeps the cached global reads: the staged form needs more
        // registers than its 16-row chunks leave, 338 against 292 us)
        constexpr bool ZSTAGE = STR && sizeof(R) == 4;
        R *ztab = (R *)(zbuf + 3 * C);
        if constexpr (ZSTAGE) {
            for (int i = t; i < C * L; i += W * C)
#pragma unroll
                for (int f = 0; f < 4; ++f) ztab[4 * i + f] = R(zr(i, f));
            __syncthreads();
        }
        auto zt = [&](int k, int f) -> R { return ZSTAGE ? ztab[4 * k + f] : R(zr(k, f)); };

        Cx<R> d[L];
        bool active;
        bool zero_lane = false;
        int q = 0, ky = 0, kyn = 0, part = 0, mm = 0;
        double s_d;  // s = -(lam_x + lam_y) dz^2 >= 0
        if (!special) {
            q = block_order(vb.x - nspecial, vb.gx - nspecial, a.reverse) * W + w;
            const int m = q % M;
            ky = q / M;
            active = (q < ny * M) && (m != 0);
            s_d = active ? -(a.lamx[m] + a.lamy[ky]) * sfac : 1.0;
            const PK_GLOBAL Cx<R> *col = S + (size_t)s * plane + (active ? q : 0);
#pragma unroll
            for (int i = 0; i < L; ++i)
                if (active && s + i < nz) {
                    const PK_GLOBAL Cx<R> &v = col[(size_t)i * plane];
                    d[i] = Cx<R>{v.re, v.im};
                } else {
                    d[i] = Cx<R>{R(0), R(0)};
                }
        } else {
            // two-mode columns: lanes [0, W/2) take part A, lanes [W/2, W) part B
            // of the same (m, ky pair), so each half reads a contiguous run of m
            // (walls along x) and the halves exchange values with a lane shuffle
            constexpr int H = W / 2 > 0 ? W / 2 : 1;
            part = w >= H ? 1 : 0;
            const int mi = w - part * H;
            const int sb = vb.x;
            const int mblk = a.xwall ? (M + H - 1) / H : 1;
            const int pair = a.xwall ? sb / mblk : sb * H + mi;
            mm = a.xwall ? (sb % mblk) * H + mi : 0;
            if (a.ywall) {
                // walls along y: the coefficients along y are real-linear, so
                // column (m, ky) holds the two real x-modes as A + iB with no
                // partner column: part A solves Re, part B solves Im
                active = pair < ny && mm < M;
                ky = active ? pair : 0;
                kyn = ky;
            } else {
                active = pair <= ny / 2 && mm < M;
                ky = active ? pair : 0;
                kyn = (ny - ky) % ny;
            }
            zero_lane = active && mm == 0 && pair == 0 && part == 0 && !a.regular;
            const double lx = a.xwall ? a.lamx[2 * (active ? mm : 0) + part]
                                      : (part ? a.lamx[M] : a.lamx[0]);
            s_d = (active && !zero_lane) ? -(lx + a.lamy[ky]) * sfac : 1.0;
            // part A reads column ky, part B column -ky (the same with walls along y)
            const PK_GLOBAL Cx<R> *col =
                S + (size_t)s * plane + (size_t)(part ? kyn : ky) * M + (active ? mm : 0);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const int k = s + i;
                Cx<R> own = {R(0), R(0)};
                if (active && k < nz) {
                    const Cx<R> g = col[(size_t)i * plane];
                    own = {g.re, g.im};
                }
                Cx<R> v;
                if (a.ywall) {
                    v = part ? Cx<R>{own.im, R(0)} : Cx<R>{own.re, R(0)};
                } else {
                    const Cx<R> oth = {__shfl_xor(own.re, H, 64), __shfl_xor(own.im, H, 64)};
                    const Cx<R> z1 = part ? oth : own;           // Z(ky)
                    const Cx<R> z2 = cconj(part ? own : oth);    // conj Z(-ky)
                    v = part ? cscale(cmul_mi(csub(z1, z2)), R(0.5)) : cscale(cadd(z1, z2), R(0.5));
                }
                d[i] = (active && k < nz) ? v : Cx<R>{R(0), R(0)};
            }
        }
#pragma unroll
        for (int i = 0; i < L; ++i)
            d[i] = cscale(d[i], R(STR ? zr(s + i, 2) * a.inv_nxny : scale));

        // zero wavenumber: raw A(0,k) = Re S[k,0,0] is re-read (L1-resident)
        // whenever needed, so the FP64 path keeps only scalars across barriers
        auto zraw = [&](int k) -> double { return double(S[(size_t)k * plane].re); };

        const R sv = R(s_d);
        const R mw = rcp_nr(R(1) + sv);  // Moebius matrix [[1, s], [1, 1+s]] / (1+s)
        const R mws = sv * mw;
        // Dirichlet walls: 2 more on the first and last pivot; row 0 maps any
        // entering v to (s + 2)/(s + 3) instead of s/(1 + s)
        const R dir2 = a.dirichlet_z ? R(2) : R(0);
        const R mws0 = a.dirichlet_z ? (sv + R(2)) * rcp_nr(sv + R(3)) : mws;

        // ---- phase 1: Moebius product of the chunk (v recurrence) -----------
        // Rows past nz (only in the last chunk) are padding: zero right-hand
        // side; v = 1 (u = 0) on row nz-1 decouples them from the real rows in
        // the back substitution, and nothing reads the last chunk's products.
        R p00 = R(1), p01 = R(0), p10 = R(0), p11 = R(1);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int k = s + i;
            R a0, b0;
            if constexpr (STR) {
                // [[a_k, s_k + D_k], [a_k, s_k + D_k + c_k]] / (s_k + D_k + c_k); a
                // row without an upper neighbour (c_k = 0) maps anything to 1
                const R ak = zt(k, 0), ck = zt(k, 1);
                const R sd = sv * zt(k, 2) + zt(k, 3);
                const R inv = rcp_nr(sd + ck);
                a0 = ck > R(0) ? ak * inv : R(0);
                b0 = ck > R(0) ? sd * inv : R(1);
            } else {
                a0 = (k == 0) ? R(0) : mw;  // row 0 ignores the entering v
                b0 = (k == 0) ? mws0 : mws;
            }
            const R n00 = a0 * p00 + b0 * p10, n01 = a0 * p01 + b0 * p11;
            const R n10 = a0 * p00 + p10, n11 = a0 * p01 + p11;
            p00 = n00; p01 = n01; p10 = n10; p11 = n11;
        }
        sl(0, c) = p00; sl(1, c) = p01; sl(2, c) = p10; sl(3, c) = p11;
        if (zero_lane) {
            double zsum = 0.0;
            for (int k = s; k < e; ++k) zsum += (STR ? zr(k, 2) : 1.0) * zraw(k);
            zbuf[c] = zsum;
        }
        __syncthreads();  // S1

        // v entering the chunk: apply the preceding chunks' maps to v (all
        // entries are >= 0 and the denominator is >= the numerator, so
        // normalising by it each step is safe and keeps the scan bounded)
        R vprev0 = R(0);
        {
            int cc = 0;
            for (; cc + 4 <= c; cc += 4) {
                R o[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int e = 0; e < 4; ++e) o[u][e] = sl(e, cc + u);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    vprev0 = (o[u][0] * vprev0 + o[u][1]) * rcp_nr(o[u][2] * vprev0 + o[u][3]);
            }
            for (; cc < c; ++cc)
                vprev0 = (sl(0, cc) * vprev0 + sl(1, cc)) * rcp_nr(sl(2, cc) * vprev0 + sl(3, cc));
        }

        // zero wavenumber, FP64: g = (raw - mean raw) * scale; face fluxes
        // F_k = sum_{j<=k} g_j; positions p_k = sum_{j<k} F_j (p_0 = 0)
        double zmu = 0.0, zF0 = 0.0, zsF = 0.0;
        if (zero_lane) {
            double tot = 0.0, pre = 0.0;
            for (int cc = 0; cc < C; ++cc) {
                if (cc == c) pre = tot;
                tot += zbuf[cc];
            }
            // stretched: the volume-weighted mean, g_k = h_k (raw_k - mean) / (nx ny),
            // and positions advance by the flux times the centre distance
            zmu = STR ? tot / a.hsum : tot / nz;
            if (c == 0 && a.zero_mean_out)
                *a.zero_mean_out = STR ? zmu * a.inv_nxny : tot * a.inv_ntot;
            zF0 = STR ? (pre - zr(s, 5) * zmu) * a.inv_nxny
                      : (pre - s * zmu) * scale;  // flux entering the chunk, F_{s-1}
            double run = zF0;
            for (int k = s; k < e; ++k) {
                run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
                zsF += STR ? run * zr(k, 4) : run;
            }
        }
        __syncthreads();  // S2: Moebius slots consumed

        // ---- phase 2: local forward elimination ------------------------------
        // Only v is kept per row: the products of u = 1 - v that carry the
        // boundary values into the chunk (G_k = u_s..u_k forward, H_k = u_k..u_e
        // backward) are rebuilt from it when needed.  Row nz-1 stores v = 1 (it
        // does not couple to the row below) and its true u separately.
        R vk[L];
        R ulast = R(0);
        {
            Cx<R> Dp = {R(0), R(0)};
            R Gp = R(1), vprev = vprev0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const int k = s + i;
                if constexpr (STR) {
                    // |pivot| = c_k + e_k, e_k = s_k + D_k + a_k v_k-1; vk holds
                    // 1/|pivot| (the multipliers are a_k / |pivot|, c_k / |pivot|)
                    const R ak = zt(k, 0), ck = zt(k, 1);
                    const R ex = sv * zt(k, 2) + zt(k, 3) + ak * vprev;
                    const R wv = rcp_nr(ck + ex);
                    const R vnew = ck > R(0) ? ex * wv : R(1);
                    Dp = cscale(csub(cscale(Dp, ak), d[i]), wv);
                    Gp = ak * wv * Gp;
                    vk[i] = wv;
                    d[i] = Dp;
                    vprev = vnew;
                } else {
                    // |pivot| = (excess over 1) + 1, except the last row (and nz = 1)
                    const R ex = (k == 0) ? sv + dir2 : sv + vprev;
                    const bool last = k >= nz - 1;
                    const R piv =
                        (nz == 1) ? sv + dir2 + dir2 : (k == nz - 1 ? ex + dir2 : R(1) + ex);
                    const R u = rcp_nr(piv);
                    const R vnew = last ? R(1) : ex * u;
                    Dp = cscale(csub(Dp, d[i]), u);
                    Gp = u * Gp;
                    if (k == nz - 1) ulast = u;
                    vk[i] = vnew;
                    d[i] = Dp;
                    vprev = vnew;
                }
            }
            sl(0, c) = Dp.re; sl(1, c) = Dp.im; sl(2, c) = Gp;
        }
        if (zero_lane) zbuf[C + c] = zsF;
        __syncthreads();  // S3

        {
            Cx<R> dprev = {R(0), R(0)};
            int cc = 0;
            for (; cc + 4 <= c; cc += 4) {
                R o[4][3];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int e = 0; e < 3; ++e) o[u][e] = sl(e, cc + u);
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    dprev = {o[u][0] + o[u][2] * dprev.re, o[u][1] + o[u][2] * dprev.im};
            }
            for (; cc < c; ++cc)
                dprev = {sl(0, cc) + sl(2, cc) * dprev.re, sl(1, cc) + sl(2, cc) * dprev.im};
            R Gr = R(1);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                Gr *= STR ? zt(s + i, 0) * vk[i] : ((s + i == nz - 1) ? ulast : R(1) - vk[i]);
                d[i] = {d[i].re + Gr * dprev.re, d[i].im + Gr * dprev.im};
            }
        }
        // ---- phase 3: local back substitution --------------------------------
        Cx<R> Xn = {R(0), R(0)};
        R Hn = R(1);
#pragma unroll
        for (int i = L - 1; i >= 0; --i) {
            // p_k = d'_k + u_k p_{k+1} written as d'_k + (p_{k+1} - v_k p_{k+1})
            Cx<R> X;
            if constexpr (STR) {
                const R uk = zt(s + i, 1) * vk[i];  // c_k / |pivot_k|
                X = {d[i].re + uk * Xn.re, d[i].im + uk * Xn.im};
                Hn *= uk;
            } else {
                X = {d[i].re + (Xn.re - vk[i] * Xn.re), d[i].im + (Xn.im - vk[i] * Xn.im)};
                Hn *= R(1) - vk[i];
            }
            d[i] = X;
            Xn = X;
        }
        double zP0 = 0.0, zsx = 0.0;
        if (zero_lane) {
            for (int cc = 0; cc < c; ++cc) zP0 += zbuf[C + cc];  // p_s
            double run = zF0, xk = zP0;
            for (int k = s; k < e; ++k) {
                zsx += STR ? zr(k, 2) * xk : xk;
                run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
                xk += STR ? run * zr(k, 4) : run;
            }
        }
        __syncthreads();  // S4: slots consumed
        sl(0, c) = Xn.re; sl(1, c) = Xn.im; sl(2, c) = Hn;
        if (zero_lane) zbuf[2 * C + c] = zsx;
        __syncthreads();  // S5

        {
            Cx<R> y = {R(0), R(0)};
            int cc = C - 1;
            for (; cc - 4 >= c; cc -= 4) {
                R o[4][3];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int e = 0; e < 3; ++e) o[u][e] = sl(e, cc - u);
#pragma unroll
                for (int u = 0; u < 4; ++u) y = {o[u][0] + o[u][2] * y.re, o[u][1] + o[u][2] * y.im};
            }
            for (; cc > c; --cc) y = {sl(0, cc) + sl(2, cc) * y.re, sl(1, cc) + sl(2, cc) * y.im};
            R Hr = R(1);
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                Hr *= STR ? zt(s + i, 1) * vk[i] : R(1) - vk[i];
                d[i] = {d[i].re + Hr * y.re, d[i].im + Hr * y.im};
            }
        }
        if (zero_lane) {
            double tot = 0.0;
            for (int cc = 0; cc < C; ++cc) tot += zbuf[2 * C + cc];
            const double mean = STR ? tot / a.hsum : tot / nz;
            double run = zF0, xk = zP0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const int k = s + i;
                if (k < nz) {
                    d[i] = {R(xk - mean), R(0)};
                    run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
                    xk += STR ? run * zr(k, 4) : run;
                }
            }
        }
        __syncthreads();  // S6: every zero-lane re-read of column (0,0) is done

        // ---- store ------------------------------------------------------------
        if (!special) {
            if (active) {
                PK_GLOBAL Cx<R> *col = S + (size_t)s * plane + q;
#pragma unroll
                for (int i = 0; i < L; ++i)
                    if (s + i < nz) col[(size_t)i * plane] = d[i];
            }
        } else {
            // the lanes of parts A and B of one (m, ky pair) are W/2 apart:
            // exchange and recombine
            constexpr int H = W / 2 > 0 ? W / 2 : 1;
            PK_GLOBAL Cx<R> *col =
                S + (size_t)s * plane + (size_t)(part == 0 ? ky : kyn) * M + (active ? mm : 0);
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const R ore = __shfl_xor(d[i].re, H, 64);
                const R oim = __shfl_xor(d[i].im, H, 64);
                const int k = s + i;
                if (active && k < nz) {
                    if (part == 0) {
                        // column ky: A + iB
                        col[(size_t)i * plane] = {d[i].re - oim, d[i].im + ore};
                    } else if (kyn != ky) {
                        // column -ky: conj(A) + i conj(B)
                        col[(size_t)i * plane] = {ore + d[i].im, -oim + d[i].re};
                    }
                }
            }
        }
    }
};

template <int W> constexpr size_t zw_lds_bytes(int C)
{
    return ((C * W * 4 * sizeof(R) + 7) / 8) * 8 + 3 * C * sizeof(double);
}

template <int L, int W, int MAXT, bool STR>
__global__ __launch_bounds__(MAXT) void k_z_walls(ZArgs a0, int C, int nspecial)
{
    extern __shared__ double smem_d[];
    ZWBody<L, W, STR>::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, C,
                           nspecial, smem_d);
}

// Walls along x and y: real systems.  Column (m, ky) of the spectrum holds
// the real coefficients of x-modes 2m and 2m+1 as its real and imaginary
// parts, and the y-modes are real as well, so viewed as reals the spectrum is
// an (nz, ny, nx) array whose entry r of row ky is the coefficient of x-mode
// r: each (r, ky) is one real tridiagonal system with
// s = -(lam_x(r) + lam_y(ky)) dz^2.  A lane takes the ZR_V = 2 adjacent
// systems r, r+1 of one row ky (nx is even): one 2-vector load per plane, a
// wavefront reads contiguous runs of 2W reals, and the recurrences of
// k_z_walls run on real values for both systems, interleaved.  The pivot
// recurrences are serial chains of reciprocals; with one system per lane
// the pass was bound by their latency (2.5 TB/s in FP64 at 512x512x256),
// two independent chains per lane keep twice the bytes in flight per chain.
// Column (0, 0) is the zero mode (FP64, as in k_z_walls): the first system
// of the first lane.
constexpr int ZR_V = 2;

template <int L, int W, int MAXT, bool STR>
__global__ __launch_bounds__(MAXT) void k_z_walls_r(ZArgs a0, int C)
{
    constexpr int V = ZR_V;
    using RV = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    if (gated_off(a0.batch, a0.gate, blockIdx.y)) return;
    ZArgs a = a0;
    if (a.batch) {
        const ProbPtrs &pq = a.batch[blockIdx.y];
        a.S = pq.S;
        if (a.zero_mean_out) a.zero_mean_out = pq.scal;
    }
    extern __shared__ double smem_d[];
    // C*W slots of 4V reals, every field lane-contiguous (zw_slot)
    R *buf = (R *)smem_d;
    double *zbuf = smem_d + ((C * W * 4 * V * sizeof(R) + 7) / 8);  // 3*C doubles

    const int t = threadIdx.x;
    const int w = t % W, c = t / W;
    auto sl = [&](int f, int cc) -> R & { return buf[zw_slot<1>(f, cc, w, C, W)]; };
    const int nz = a.nz, nx = a.nx, ny = a.ny;
    const size_t plane = (size_t)ny * nx;  // reals per z-plane
    PK_GLOBAL R *S = gbl((R *)a.S);
    const int s = c * L;
    const int e = (s + L < nz) ? s + L : nz;  // chunk rows [s, e)
    const double scale = a.dz2 * a.inv_nxny;
    // stretched z: row coefficients from the table, s per row times h_k (as
    // in ZWBody)
    const double *zrow = a.zrow;
    auto zr = [&](int k, int f) -> double { return zrow[8 * k + f]; };
    const double sfac = STR ? 1.0 : a.dz2;
    // stretched rows staged in LDS in FP32 (as in ZWBody)
    constexpr bool ZSTAGE = STR && sizeof(R) == 4;
    R *ztab = (R *)(zbuf + 3 * C);
    if constexpr (ZSTAGE) {
        for (int i = t; i < C * L; i += W * C)
#pragma unroll
            for (int f = 0; f < 4; ++f) ztab[4 * i + f] = R(zr(i, f));
        __syncthreads();
    }
    auto zt = [&](int k, int f) -> R { return ZSTAGE ? ztab[4 * k + f] : R(zr(k, f)); };

    // systems q0 + v, v < V, of row ky
    const int q0 = (block_order((int)blockIdx.x, (int)gridDim.x, a.reverse) * W + w) * V;
    const int r0 = q0 % nx, ky = q0 / nx;
    const bool active = q0 < ny * nx;
    const bool zero_lane = active && q0 == 0 && !a.regular;
    const R dir2 = a.dirichlet_z ? R(2) : R(0);
    R sv[V], mw[V], mws[V], mws0[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const bool zcol = zero_lane && v == 0;
        const double s_d = (active && !zcol) ? -(a.lamx[r0 + v] + a.lamy[ky]) * sfac : 1.0;
        sv[v] = R(s_d);
        mw[v] = rcp_nr(R(1) + sv[v]);
        mws[v] = sv[v] * mw[v];
        mws0[v] = a.dirichlet_z ? (sv[v] + R(2)) * rcp_nr(sv[v] + R(3)) : mws[v];
    }

    R d[L][V];
    {
        const PK_GLOBAL R *col = S + (size_t)s * plane + (active ? q0 : 0);
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const R sc = R(STR ? zr(s + i, 2) * a.inv_nxny : scale);
            RV x{R(0), R(0)};
            if (active && s + i < nz) x = *(const PK_GLOBAL RV *)(col + (size_t)i * plane);
            d[i][0] = x.x * sc;
            d[i][1] = x.y * sc;
        }
    }
    // zero wavenumber: raw values re-read (L1-resident) whenever needed
    auto zraw = [&](int k) -> double { return double(S[(size_t)k * plane]); };

    // ---- phase 1: Moebius product of the chunk (v recurrence) -----------
    R p00[V], p01[V], p10[V], p11[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        p00[v] = R(1); p01[v] = R(0); p10[v] = R(0); p11[v] = R(1);
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int k = s + i;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            R x0, y0;
            if constexpr (STR) {
                const R ak = zt(k, 0), ck = zt(k, 1);
                const R sd = sv[v] * zt(k, 2) + zt(k, 3);
                const R inv = rcp_nr(sd + ck);
                x0 = ck > R(0) ? ak * inv : R(0);
                y0 = ck > R(0) ? sd * inv : R(1);
            } else {
                x0 = (k == 0) ? R(0) : mw[v];
                y0 = (k == 0) ? mws0[v] : mws[v];
            }
            const R n00 = x0 * p00[v] + y0 * p10[v], n01 = x0 * p01[v] + y0 * p11[v];
            const R n10 = x0 * p00[v] + p10[v], n11 = x0 * p01[v] + p11[v];
            p00[v] = n00; p01[v] = n01; p10[v] = n10; p11[v] = n11;
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sl(4 * v, c) = p00[v]; sl(4 * v + 1, c) = p01[v]; sl(4 * v + 2, c) = p10[v]; sl(4 * v + 3, c) = p11[v];
    }
    if (zero_lane) {
        double zsum = 0.0;
        for (int k = s; k < e; ++k) zsum += (STR ? zr(k, 2) : 1.0) * zraw(k);
        zbuf[c] = zsum;
    }
    __syncthreads();  // S1

    R vprev0[V];
#pragma unroll
    for (int v = 0; v < V; ++v) vprev0[v] = R(0);
    {
        int cc = 0;
        for (; cc + 2 <= c; cc += 2) {
            R o[2][4 * V];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int j = 0; j < 4 * V; ++j) o[u][j] = sl(j, cc + u);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const R *q = o[u] + 4 * v;
                    vprev0[v] = (q[0] * vprev0[v] + q[1]) * rcp_nr(q[2] * vprev0[v] + q[3]);
                }
        }
        for (; cc < c; ++cc) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                vprev0[v] = (sl(4 * v, cc) * vprev0[v] + sl(4 * v + 1, cc)) *
                            rcp_nr(sl(4 * v + 2, cc) * vprev0[v] + sl(4 * v + 3, cc));
        }
    }

    double zmu = 0.0, zF0 = 0.0, zsF = 0.0;
    if (zero_lane) {
        double tot = 0.0, pre = 0.0;
        for (int cc = 0; cc < C; ++cc) {
            if (cc == c) pre = tot;
            tot += zbuf[cc];
        }
        zmu = STR ? tot / a.hsum : tot / nz;
        if (c == 0 && a.zero_mean_out)
            *a.zero_mean_out = STR ? zmu * a.inv_nxny : tot * a.inv_ntot;
        zF0 = STR ? (pre - zr(s, 5) * zmu) * a.inv_nxny : (pre - s * zmu) * scale;
        double run = zF0;
        for (int k = s; k < e; ++k) {
            run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
            zsF += STR ? run * zr(k, 4) : run;
        }
    }
    __syncthreads();  // S2

    // ---- phase 2: local forward elimination ------------------------------
    R vk[L][V];
    R ulast[V], Dp[V], Gp[V], vprev[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        ulast[v] = R(0); Dp[v] = R(0); Gp[v] = R(1); vprev[v] = vprev0[v];
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const int k = s + i;
#pragma unroll
        for (int v = 0; v < V; ++v) {
            if constexpr (STR) {
                // vk holds 1/|pivot| (as in ZWBody)
                const R ak = zt(k, 0), ck = zt(k, 1);
                const R ex = sv[v] * zt(k, 2) + zt(k, 3) + ak * vprev[v];
                const R wv = rcp_nr(ck + ex);
                const R vnew = ck > R(0) ? ex * wv : R(1);
                Dp[v] = (ak * Dp[v] - d[i][v]) * wv;
                Gp[v] = ak * wv * Gp[v];
                vk[i][v] = wv;
                d[i][v] = Dp[v];
                vprev[v] = vnew;
            } else {
                const R ex = (k == 0) ? sv[v] + dir2 : sv[v] + vprev[v];
                const bool last = k >= nz - 1;
                const R piv = (nz == 1) ? sv[v] + dir2 + dir2 : (k == nz - 1 ? ex + dir2 : R(1) + ex);
                const R u = rcp_nr(piv);
                const R vnew = last ? R(1) : ex * u;
                Dp[v] = (Dp[v] - d[i][v]) * u;
                Gp[v] = u * Gp[v];
                if (k == nz - 1) ulast[v] = u;
                vk[i][v] = vnew;
                d[i][v] = Dp[v];
                vprev[v] = vnew;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sl(4 * v, c) = Dp[v];
        sl(4 * v + 1, c) = Gp[v];
    }
    if (zero_lane) zbuf[C + c] = zsF;
    __syncthreads();  // S3

    {
        R dprev[V];
#pragma unroll
        for (int v = 0; v < V; ++v) dprev[v] = R(0);
        for (int cc = 0; cc < c; ++cc)
#pragma unroll
            for (int v = 0; v < V; ++v) dprev[v] = sl(4 * v, cc) + sl(4 * v + 1, cc) * dprev[v];
        R Gr[V];
#pragma unroll
        for (int v = 0; v < V; ++v) Gr[v] = R(1);
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                Gr[v] *= STR ? zt(s + i, 0) * vk[i][v]
                             : ((s + i == nz - 1) ? ulast[v] : R(1) - vk[i][v]);
                d[i][v] = d[i][v] + Gr[v] * dprev[v];
            }
    }
    // ---- phase 3: local back substitution --------------------------------
    R Xn[V], Hn[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        Xn[v] = R(0); Hn[v] = R(1);
    }
#pragma unroll
    for (int i = L - 1; i >= 0; --i)
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const R uk = STR ? zt(s + i, 1) * vk[i][v] : R(1) - vk[i][v];
            const R X = STR ? d[i][v] + uk * Xn[v] : d[i][v] + (Xn[v] - vk[i][v] * Xn[v]);
            d[i][v] = X;
            Xn[v] = X;
            Hn[v] *= uk;
        }
    double zP0 = 0.0, zsx = 0.0;
    if (zero_lane) {
        for (int cc = 0; cc < c; ++cc) zP0 += zbuf[C + cc];
        double run = zF0, xk = zP0;
        for (int k = s; k < e; ++k) {
            zsx += STR ? zr(k, 2) * xk : xk;
            run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
            xk += STR ? run * zr(k, 4) : run;
        }
    }
    __syncthreads();  // S4
#pragma unroll
    for (int v = 0; v < V; ++v) {
        sl(4 * v, c) = Xn[v];
        sl(4 * v + 1, c) = Hn[v];
    }
    if (zero_lane) zbuf[2 * C + c] = zsx;
    __syncthreads();  // S5

    {
        R y[V];
#pragma unroll
        for (int v = 0; v < V; ++v) y[v] = R(0);
        for (int cc = C - 1; cc > c; --cc)
#pragma unroll
            for (int v = 0; v < V; ++v) y[v] = sl(4 * v, cc) + sl(4 * v + 1, cc) * y[v];
        R Hr[V];
#pragma unroll
        for (int v = 0; v < V; ++v) Hr[v] = R(1);
#pragma unroll
        for (int i = L - 1; i >= 0; --i)
#pragma unroll
            for (int v = 0; v < V; ++v) {
                Hr[v] *= STR ? zt(s + i, 1) * vk[i][v] : R(1) - vk[i][v];
                d[i][v] = d[i][v] + Hr[v] * y[v];
            }
    }
    if (zero_lane) {
        double tot = 0.0;
        for (int cc = 0; cc < C; ++cc) tot += zbuf[2 * C + cc];
        const double mean = STR ? tot / a.hsum : tot / nz;
        double run = zF0, xk = zP0;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int k = s + i;
            if (k < nz) {
                d[i][0] = R(xk - mean);
                run += STR ? zr(k, 2) * (zraw(k) - zmu) * a.inv_nxny : (zraw(k) - zmu) * scale;
                xk += STR ? run * zr(k, 4) : run;
            }
        }
    }
    __syncthreads();  // S6: every zero-lane re-read of column (0,0) is done

    if (active) {
        PK_GLOBAL R *col = S + (size_t)s * plane + q0;
#pragma unroll
        for (int i = 0; i < L; ++i)
            if (s + i < nz) *(PK_GLOBAL RV *)(col + (size_t)i * plane) = RV{d[i][0], d[i][1]};
    }
}

// W lanes (2W systems) per chunk row; workgroup size limits that leave the
// registers the chunks hold (FP32: 16-row chunks at most 512 threads, 8-row
// chunks 1024; FP64 half of that)
template <int L> constexpr int zwr_maxt() { return (L == 16 ? 512 : 1024) / (sizeof(R) == 8 ? 2 : 1); }

template <int L, int W, bool STR>
static int run_zwr(const ZArgs &a, hipStream_t s)
{
    constexpr int MAXT = zwr_maxt<L>();
    const int C = (a.nz + L - 1) / L;
    if (C * W > MAXT || a.nx % ZR_V != 0) return -1;
    const int nb = (a.ny * a.nx / ZR_V + W - 1) / W;
    const size_t shm = ((C * W * 4 * ZR_V * sizeof(R) + 7) / 8) * 8 + 3 * C * sizeof(double) +
                       (STR && sizeof(R) == 4 ? (size_t)C * L * 4 * sizeof(R) : 0);
    hipLaunchKernelGGL((k_z_walls_r<L, W, MAXT, STR>), dim3(nb, a.batch ? a.nbatch : 1),
                       dim3(W * C), shm, s, a, C);
    return (int)hipGetLastError();
}

template <int L, int W, int MAXT, bool STR>
static int run_zw(const ZArgs &a, hipStream_t s)
{
    const int C = (a.nz + L - 1) / L;
    if (C * W > MAXT) return -1;
    const int npairs = a.ywall ? a.ny : a.ny / 2 + 1;
    constexpr int H = W / 2 > 0 ? W / 2 : 1;
    const int nspecial = a.xwall ? npairs * ((a.M + H - 1) / H) : (npairs + H - 1) / H;
    const int nmain = a.xwall ? 0 : (a.ny * a.M + W - 1) / W;
    const size_t shm = ((C * W * 4 * sizeof(R) + 7) / 8) * 8 + 3 * C * sizeof(double) +
                       (STR && sizeof(R) == 4 ? (size_t)C * L * 4 * sizeof(R) : 0);
    hipLaunchKernelGGL((k_z_walls<L, W, MAXT, STR>), dim3(nspecial + nmain, a.batch ? a.nbatch : 1),
                       dim3(W * C), shm, s, a, C, nspecial);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work list: the z passes of problems of different shapes and z boundaries in
// one launch.  Classes: 1 walls with nz <= 64 (8-row chunks, 32 columns per
// workgroup), 2 walls with nz <= 256 (16-row chunks, 128-byte row runs), and
// 1000 + N periodic columns of length N (the FFT body of k_zperiodic.hip).
// Boxes with walls along both x and y keep their own launch.
// ---------------------------------------------------------------------------
#include "zper_body.hpp"

constexpr int ZL_NT = 256;
constexpr int ZL_W2 = 128 / (int)sizeof(Cx<R>);
#define PK_ZL_LENGTHS(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

// SHORT: only columns of 64 rows or fewer (classes 1 and 1000 + N, N <= 64),
// which need far fewer registers than the 16-row chunks of class 2
template <bool SHORT>
__global__ __launch_bounds__(ZL_NT) void k_z_list(ListArgs<ZArgs>)
{
    extern __shared__ double smem_d[];
    const PK_KARG ListArgs<ZArgs> *L = list_args<ZArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const ZArgs arg = L->a[g];
    switch (L->cls[g]) {
    case 1: ZWBody<8, 32>::run(arg, vb, L->aux[g], L->aux2[g], smem_d); break;
    case 2:
        if constexpr (!SHORT) ZWBody<16, ZL_W2>::run(arg, vb, L->aux[g], L->aux2[g], smem_d);
        break;
#define PK_ZL_CASE(N)                                                                         \
    case 1000 + N:                                                                            \
        if constexpr (ZPCfg<N>::NT <= ZL_NT && (!SHORT || N <= 64))                           \
            ZPBody<N>::run(arg, vb, L->aux2[g], (char *)smem_d);                              \
        break;
        PK_ZL_LENGTHS(PK_ZL_CASE)
#undef PK_ZL_CASE
    default: break;
    }
}

// class, threads, blocks per problem, chunks, special blocks and LDS of a z
// record in the list kernel; false when it has no class there
static bool z_list_class(const ZArgs &a, int &cls, int &nt, int &gx, int &C, int &nspecial,
                         size_t &lds)
{
    if (!a.periodic_z) {
        if ((a.xwall && a.ywall) || a.zrow) return false;
        int L, W;
        if (a.nz <= 64) {
            cls = 1; L = 8; W = 32;
        } else if (a.nz <= 256) {
            cls = 2; L = 16; W = ZL_W2;
        } else {
            return false;
        }
        C = (a.nz + L - 1) / L;
        nt = W * C;
        if (nt > ZL_NT) return false;
        const int npairs = a.ywall ? a.ny : a.ny / 2 + 1;
        const int H = W / 2 > 0 ? W / 2 : 1;
        nspecial = a.xwall ? npairs * ((a.M + H - 1) / H) : (npairs + H - 1) / H;
        const int nmain = a.xwall ? 0 : (a.ny * a.M + W - 1) / W;
        gx = nspecial + nmain;
        lds = cls == 1 ? zw_lds_bytes<32>(C) : zw_lds_bytes<ZL_W2>(C);
        return true;
    }
    switch (a.nz) {
#define PK_ZL_INFO(N)                                                                   \
    case N: {                                                                           \
        using Cf = ZPCfg<N>;                                                            \
        if (Cf::NT > ZL_NT) return false;                                               \
        constexpr int NB = Cf::NB, NP = Cf::NB / 2;                                     \
        const int npairs = a.ny / 2 + 1;                                                \
        int nmain = (a.ny * a.M + NB - 1) / NB;                                         \
        if (a.xwall) {                                                                  \
            nspecial = a.ywall ? a.ny * ((a.M + NB - 1) / NB) : npairs * ((a.M + NP - 1) / NP); \
            nmain = 0;                                                                  \
        } else {                                                                        \
            nspecial = a.ywall ? (a.ny + NB - 1) / NB : (npairs + NP - 1) / NP;         \
        }                                                                               \
        cls = 1000 + N;                                                                 \
        nt = Cf::NT;                                                                    \
        gx = nspecial + nmain;                                                          \
        C = 0;                                                                          \
        lds = ZPBody<N>::LDS_BYTES;                                                     \
        return true;                                                                    \
    }
        PK_ZL_LENGTHS(PK_ZL_INFO)
#undef PK_ZL_INFO
    default: return false;
    }
}

}  // namespace PK_NS
using namespace PK_NS;

int PK_SUFFIX(launch_z_walls)(const ZArgs &a, hipStream_t s);
int PK_SUFFIX(launch_z_periodic)(const ZArgs &a, hipStream_t s);

int PK_SUFFIX(launch_z_list)(const ZArgs *a, int n, hipStream_t s)
{
    ListArgs<ZArgs> L{};
    size_t lds = 0;
    int total = 0;
    bool shorts = true;  // every segment has columns of 64 rows or fewer
    auto flush = [&]() -> int {
        if (L.nseg == 0) return 0;
        L.start[L.nseg] = total;
        if (shorts)
            hipLaunchKernelGGL(k_z_list<true>, dim3(total), dim3(ZL_NT), lds, s, L);
        else
            hipLaunchKernelGGL(k_z_list<false>, dim3(total), dim3(ZL_NT), lds, s, L);
        L.nseg = 0;
        total = 0;
        lds = 0;
        shorts = true;
        return (int)hipGetLastError();
    };
    for (int i = 0; i < n; ++i) {
        int cls = 0, nt = 0, gx = 0, C = 0, nsp = 0;
        size_t b = 0;
        if (!z_list_class(a[i], cls, nt, gx, C, nsp, b)) {
            const int e = a[i].periodic_z ? PK_SUFFIX(launch_z_periodic)(a[i], s)
                                          : PK_SUFFIX(launch_z_walls)(a[i], s);
            if (e) return e;
            continue;
        }
        const int g = L.nseg++;
        L.start[g] = total;
        L.gx[g] = gx;
        L.cls[g] = cls;
        L.nt[g] = nt;
        L.aux[g] = C;
        L.aux2[g] = nsp;
        L.a[g] = a[i];
        shorts = shorts && a[i].nz <= 64;
        total += gx * (a[i].batch ? a[i].nbatch : 1);
        lds = lds > b ? lds : b;
        if (L.nseg == LIST_MAX_SEG) {
            const int e = flush();
            if (e) return e;
        }
    }
    return flush();
}

namespace PK_NS {
// tile choice of the wall-bounded z solve; STR: stretched rows (ZArgs::zrow)
template <bool STR> static int dispatch_zw(const ZArgs &a, hipStream_t s)
{
    // Chunk length L (registers per thread), W columns per workgroup,
    // W*ceil(nz/L) threads.  a.variant selects the tile (autotuned per shape):
    //   0: 16-row chunks, 128-byte row runs (W = 16 FP32 / 8 FP64)
    //   1: 8-row chunks (fewer registers, longer cross-chunk scans)
    //   2: 16-row chunks, 256-byte row runs (W = 32 FP32 / 16 FP64)
    //   3: 8-row chunks, 256-byte row runs
    const int nz = a.nz;
    constexpr bool F32 = sizeof(R) == 4;
    if (a.xwall && a.ywall) {
        // every column holds two real modes: real systems, two per lane
        // (k_z_walls_r).  Tiles as below: 16- or 8-row chunks, 128- or
        // 256-byte row runs, narrowed to fit the workgroup size limit (deep
        // grids take 8-row chunks)
        const int v = a.variant & 3;
        int L = (v == 1 || v == 3 || nz > 1024) ? 8 : 16;
        int W = (F32 ? 16 : 8) * (v >= 2 ? 2 : 1);
        const int maxt = L == 16 ? zwr_maxt<16>() : zwr_maxt<8>();
        const int C = (nz + L - 1) / L;
        while (W > 1 && C * W > maxt) W /= 2;
        // shallow grids: wider workgroups
        while (W < 32 && C * W < 256 && 2 * C * W <= maxt) W *= 2;
        if (L == 16) {
            switch (W) {
            case 32: return run_zwr<16, 32, STR>(a, s);
            case 16: return run_zwr<16, 16, STR>(a, s);
            case 8: return run_zwr<16, 8, STR>(a, s);
            case 4: return run_zwr<16, 4, STR>(a, s);
            default: return -1;
            }
        }
        switch (W) {
        case 32: return run_zwr<8, 32, STR>(a, s);
        case 16: return run_zwr<8, 16, STR>(a, s);
        case 8: return run_zwr<8, 8, STR>(a, s);
        case 4: return run_zwr<8, 4, STR>(a, s);
        case 2: return run_zwr<8, 2, STR>(a, s);
        case 1: return run_zwr<8, 1, STR>(a, s);
        default: return -1;
        }
    }
    const bool c8 = a.variant == 1 || a.variant == 3;
    // walls along x: every column is a two-mode column whose lane halves
    // read W/2 consecutive m each, so only the wide tiles give full
    // 128-byte runs (narrow ones split cache lines across dies)
    const bool wide = a.variant >= 2 || a.xwall;
    if (nz <= 64) return run_zw<8, 32, 256, STR>(a, s);
    if (!c8) {
        if constexpr (F32) {
            if (wide) {
                if (nz <= 128) return run_zw<16, 32, 256, STR>(a, s);
                if (nz <= 256) return run_zw<16, 32, 512, STR>(a, s);
                if (nz <= 512) return run_zw<16, 32, 1024, STR>(a, s);
            } else {
                if (nz <= 256) return run_zw<16, 16, 256, STR>(a, s);
                if (nz <= 512) return run_zw<16, 16, 512, STR>(a, s);
                if (nz <= 1024) return run_zw<16, 16, 1024, STR>(a, s);
            }
            if (nz <= 4096) return run_zw<16, 2, 1024, STR>(a, s);
        } else {
            if (wide) {
                if (nz <= 256) return run_zw<16, 16, 256, STR>(a, s);
                if (nz <= 512) return run_zw<16, 16, 512, STR>(a, s);
            } else {
                if (nz <= 512) return run_zw<16, 8, 256, STR>(a, s);
                if (nz <= 1024) return run_zw<16, 8, 512, STR>(a, s);
            }
        }
    }
    if (wide && !F32) {
        if (nz <= 256) return run_zw<8, 16, 512, STR>(a, s);
        if (nz <= 512) return run_zw<8, 16, 1024, STR>(a, s);
    }
    if (wide && F32) {
        if (nz <= 256) return run_zw<8, 32, 1024, STR>(a, s);
    }
    if (nz <= 512) return run_zw<8, 8, 512, STR>(a, s);
    if (nz <= 1024) return run_zw<8, 8, 1024, STR>(a, s);
    if (nz <= 4096) return run_zw<8, 2, 1024, STR>(a, s);
    return -1;
}
}  // namespace PK_NS

int PK_SUFFIX(launch_z_walls)(const ZArgs &a, hipStream_t s)
{
    return a.zrow ? dispatch_zw<true>(a, s) : dispatch_zw<false>(a, s);
}

}  // namespace pk
