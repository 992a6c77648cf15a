// k_misc.hip -- precision dispatch of the pass launchers and the
// deterministic FP64 reduction of per-workgroup partial sums (residual and
// right-hand-side norms of the iterative refinement).
#include "../../include/poisson.h"
#include "common.hpp"
#include "lengths.hpp"
#include "stencil.hpp"

namespace pk {

int launch_x_fwd_f32(const XFwdArgs &, hipStream_t, int *);
int launch_x_fwd_f64(const XFwdArgs &, hipStream_t, int *);
int launch_x_inv_f32(const XInvArgs &, hipStream_t);
int launch_x_inv_f64(const XInvArgs &, hipStream_t);
int launch_y_f32(const YArgs &, hipStream_t);
int launch_y_f64(const YArgs &, hipStream_t);
int launch_z_walls_f32(const ZArgs &, hipStream_t);
int launch_z_walls_f64(const ZArgs &, hipStream_t);
int launch_z_periodic_f32(const ZArgs &, hipStream_t);
int launch_z_periodic_f64(const ZArgs &, hipStream_t);
int x_fwd_blocks_f32(int, int, int, int, int, int);
int x_fwd_blocks_f64(int, int, int, int, int, int);
int x_res_slots_f32(int, int, int);
int launch_y_list_f32(const YArgs *, int, hipStream_t);
int launch_y_list_f64(const YArgs *, int, hipStream_t);
int launch_z_list_f32(const ZArgs *, int, hipStream_t);
int launch_z_list_f64(const ZArgs *, int, hipStream_t);
int launch_x_fwd_list_f32(const XFwdArgs *, int, hipStream_t);
int launch_x_fwd_list_f64(const XFwdArgs *, int, hipStream_t);
int launch_x_inv_list_f32(const XInvArgs *, int, hipStream_t);
int launch_x_inv_list_f64(const XInvArgs *, int, hipStream_t);
int x_fwd_list_blocks_f32(const XFwdArgs &);
int x_fwd_list_blocks_f64(const XFwdArgs &);

int launch_y_list(int prec, const YArgs *a, int n, hipStream_t s)
{
    return prec == P_F32 ? launch_y_list_f32(a, n, s) : launch_y_list_f64(a, n, s);
}
int launch_z_list(int prec, const ZArgs *a, int n, hipStream_t s)
{
    return prec == P_F32 ? launch_z_list_f32(a, n, s) : launch_z_list_f64(a, n, s);
}
int launch_x_fwd_list(int prec, const XFwdArgs *a, int n, hipStream_t s)
{
    return prec == P_F32 ? launch_x_fwd_list_f32(a, n, s) : launch_x_fwd_list_f64(a, n, s);
}
int launch_x_inv_list(int prec, const XInvArgs *a, int n, hipStream_t s)
{
    return prec == P_F32 ? launch_x_inv_list_f32(a, n, s) : launch_x_inv_list_f64(a, n, s);
}
int x_fwd_list_blocks(int prec, const XFwdArgs &a)
{
    return prec == P_F32 ? x_fwd_list_blocks_f32(a) : x_fwd_list_blocks_f64(a);
}

int launch_x_fwd(int prec, const XFwdArgs &a, int *nblocks_out, hipStream_t s)
{
    return prec == P_F32 ? launch_x_fwd_f32(a, s, nblocks_out) : launch_x_fwd_f64(a, s, nblocks_out);
}
int launch_x_inv(int prec, const XInvArgs &a, hipStream_t s)
{
    return prec == P_F32 ? launch_x_inv_f32(a, s) : launch_x_inv_f64(a, s);
}
int launch_y(int prec, const YArgs &a, hipStream_t s)
{
    return prec == P_F32 ? launch_y_f32(a, s) : launch_y_f64(a, s);
}
int launch_z_walls(int prec, const ZArgs &a, hipStream_t s)
{
    return prec == P_F32 ? launch_z_walls_f32(a, s) : launch_z_walls_f64(a, s);
}
int launch_z_periodic(int prec, const ZArgs &a, hipStream_t s)
{
    return prec == P_F32 ? launch_z_periodic_f32(a, s) : launch_z_periodic_f64(a, s);
}
int x_fwd_blocks(int prec, int nx, int ny, int nz, int residual, int kr_max, int kr_nb)
{
    return prec == P_F32 ? x_fwd_blocks_f32(nx, ny, nz, residual, kr_max, kr_nb)
                         : x_fwd_blocks_f64(nx, ny, nz, residual, kr_max, kr_nb);
}

#define PK_IS(N) case N: return true;
bool fft_length_supported(int n)
{
    switch (n) { PK_LENGTHS(PK_IS) default: return false; }
}

// Sum of the three sums of n partial records (stride 4 doubles): thread t
// adds records t, t+1024, ... in a fixed order, then a fixed-shape tree
// finishes; bitwise reproducible for a given n.  Every thread gets the totals.
__device__ __forceinline__ void sum_records(const double *in_, int n, double (*sh)[1024],
                                            double &s0, double &s1, double &s2)
{
    const int t = threadIdx.x;
    const PK_GLOBAL double *in = gbl(in_);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = t; i < n; i += 1024) {
        const double4 v = *(const PK_GLOBAL double4 *)(in + 4 * (size_t)i);
        a0 += v.x;
        a1 += v.y;
        a2 += v.z;
    }
    sh[0][t] = a0;
    sh[1][t] = a1;
    sh[2][t] = a2;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h) {
            sh[0][t] += sh[0][t + h];
            sh[1][t] += sh[1][t + h];
            sh[2][t] += sh[2][t + h];
        }
        __syncthreads();
    }
    s0 = sh[0][0];
    s1 = sh[1][0];
    s2 = sh[2][0];
}

// Refinement control (device-side loop): opening a loop, and the decision
// after a residual evaluation with the host-driven loop's rules:
//   rho = ||r|| / ||f - mean f||;  rho <= rtol -> converged;  non-finite ->
//   error;  max_refine corrections done, or rho > rho_prev / 2 (stall) ->
//   not converged; otherwise correct, and when rho_prev * rho_first is two
//   decades below rtol the next residual is evaluated without transform.
__device__ __forceinline__ void ctrl_open(int *c, double *sc)
{
    c[C_STATE] = 1;
    c[C_FULL] = 1;
    c[C_CHECK] = 0;
    c[C_EVAL] = 1;
    c[C_FIX] = 0;
    c[C_CORRECT] = 0;
    c[C_CORR] = 0;
    c[C_STATUS] = POISSON_OK;
    c[C_COPY] = 0;
    sc[5] = -1.0;
    sc[6] = -1.0;
    sc[7] = -1.0;
}

__device__ __forceinline__ void ctrl_decide(int *c, double *sc, double rtol, int max_refine)
{
    const bool was_check = c[C_CHECK] != 0;
    const double rho = sc[3] > 0.0 ? sqrt(sc[2] / sc[3]) : sqrt(sc[2]);
    sc[5] = rho;
    if (sc[7] < 0.0) sc[7] = rho;
    int status = 1;  // 1: go on
    if (!isfinite(rho))
        status = POISSON_ERR_NONFINITE;
    else if (rho <= rtol)
        status = POISSON_OK;
    else if (c[C_CORR] >= max_refine || (sc[6] >= 0.0 && rho > 0.5 * sc[6]))
        status = POISSON_ERR_NOT_CONVERGED;
    if (status != 1) {
        c[C_STATUS] = status;
        c[C_STATE] = 0;
        c[C_FULL] = c[C_CHECK] = c[C_EVAL] = c[C_FIX] = c[C_CORRECT] = 0;
        c[C_COPY] = c[C_CORR] == 0 ? 1 : 0;
        return;
    }
    sc[6] = rho;
    c[C_CORR] += 1;
    c[C_FIX] = was_check ? 1 : 0;
    c[C_CORRECT] = 1;
    const bool predict = sc[7] > 0.0 && sc[6] > 0.0 && sc[6] * sc[7] * 100.0 <= rtol;
    c[C_FULL] = predict ? 0 : 1;
    c[C_CHECK] = predict ? 1 : 0;
    c[C_EVAL] = 1;
}

// One workgroup per problem: the sums of the partial records into
// out[0..3) (batched: scal + out_off of problem blockIdx.x), then, by mode,
// nothing (0), opening the control record (1) or the control decision (2).
__global__ __launch_bounds__(1024) void k_sum_partials(const double *in, int n, double *out,
                                                       const ProbPtrs *batch, int out_off,
                                                       int gate, int mode, double rtol,
                                                       int max_refine, int n_check)
{
    __shared__ double sh[3][1024];
    if (gated_off(batch, gate, blockIdx.x)) return;
    if (batch) {
        in = batch[blockIdx.x].partials;
        out = batch[blockIdx.x].scal + out_off;
    }
    // after a residual evaluation: records of the check pass, or of the
    // residual pass with transform (their grids differ)
    if (mode == 2 && batch[blockIdx.x].ctrl[C_CHECK]) n = n_check;
    double s0, s1, s2;
    sum_records(in, n, sh, s0, s1, s2);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
        if (mode == 1) ctrl_open(batch[blockIdx.x].ctrl, batch[blockIdx.x].scal);
        if (mode == 2) ctrl_decide(batch[blockIdx.x].ctrl, batch[blockIdx.x].scal, rtol, max_refine);
    }
}

int launch_sum_partials(const double *in, int n, double *out, const ProbPtrs *batch,
                        int nbatch, int out_off, hipStream_t s, int gate, int mode, double rtol,
                        int max_refine, int n_check)
{
    if (mode != 0 && !batch) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sum_partials, dim3(batch ? nbatch : 1), dim3(1024), 0, s, in, n, out,
                       batch, out_off, gate, mode, rtol, max_refine, n_check);
    return (int)hipGetLastError();
}

// Residual of the discrete equation, r = (f - mean f) - L p, in FP64 (the
// 7-point operator of the marker-and-cell grid, 2.5-D march of stencil.hpp):
// streams f and p once and writes three partial sums per workgroup: sum r^2,
// sum (f - mean f)^2, sum p.  512 threads share a plane tile of about 2048
// pairs (4 per thread): 118 VGPRs and four waves per SIMD at nx = 512, where
// 256 threads (8 pairs each) needed 200 and ran two (212 -> 207 us at
// 512x512x256).
constexpr int RC_NT = 512;

// One workgroup's work (plane range and row block vb.x of problem vb.y);
// LDS carved from `lds` (LDS_BYTES).
template <int M> struct RCBody {
    static constexpr int TJ = march_rows(M);
    using Mar = PlaneMarch<M, TJ, RC_NT>;
    static constexpr size_t TILE_B = sizeof(double2) * (TJ + 2) * M;
    static constexpr size_t LDS_BYTES = TILE_B + sizeof(double) * 3 * (RC_NT / 64);

    static __device__ __forceinline__ void run(const XFwdArgs &a0, VBlock vb, char *lds)
    {

        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        double2(*s_tile)[M] = (double2(*)[M])lds;
        double *s_red = (double *)(lds + TILE_B);
        XFwdArgs a = a0;
        if (a.batch) {
            const ProbPtrs &q = a.batch[vb.y];
            a.f = q.f;
            a.p = q.p;
            a.partials = q.partials;
            a.sum_f = q.scal + 1;
        }
        const int njb = march_jblocks(a.ny, TJ);
        const int bid = block_order(xcd_order(vb.x, vb.gx), vb.gx, a.reverse);
        const int jb = bid % njb, kb = bid / njb;
        const int kr = march_planes(a.ny, a.nz, TJ, a.kr_max, a.kr_nb);
        const int k0 = kb * kr;
        const int k1 = k0 + kr < a.nz ? k0 + kr : a.nz;
        Mar m;
        m.f = gbl(a.f);
        m.p = gbl(a.p);
        m.ax = a.ax;
        m.ay = a.ay;
        m.az = a.az;
        m.zc = a.zc;
        m.mu = (a.sum_f && !a.regular) ? (*a.sum_f) * a.inv_n : 0.0;
        m.tile = s_tile;
        m.setup(jb, a.ny, a.nz, a.bc_z, a.bc_y);
        m.bc_x = a.bc_x;
        m.start(k0);
        double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
        double wk = 1.0;  // stretched z: volume weight of p in plane k
        auto sink = [&](int, int, int, double r0, double r1, double f0, double f1, double2 c) {
            acc0 += r0 * r0 + r1 * r1;
            acc1 += f0 * f0 + f1 * f1;
            acc2 += wk * (c.x + c.y);
        };
        for (int k = k0; k < k1; ++k) {
            if (k > k0) __syncthreads();
            wk = a.hz ? a.hz[k] : 1.0;
            m.fetch(k);
            m.step(k, sink);
        }
        block_sum3(acc0, acc1, acc2, s_red, RC_NT);
        if (threadIdx.x == 0) {
            a.partials[4 * vb.x] = acc0;
            a.partials[4 * vb.x + 1] = acc1;
            a.partials[4 * vb.x + 2] = acc2;
        }
    }
};

template <int M>
__global__ __launch_bounds__(RC_NT) void k_residual_check(XFwdArgs a0)
{
    using B = RCBody<M>;
    __shared__ __align__(16) char s_lds[B::LDS_BYTES];
    B::run(a0, VBlock{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x}, s_lds);
}

template <int M> static int rc_blocks(int ny, int nz, int kr_max, int kr_nb)
{
    return march_jblocks(ny, march_rows(M)) *
           march_kblocks(ny, nz, march_rows(M), kr_max, kr_nb);
}

template <int M> static int run_rc(const XFwdArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_residual_check<M>,
                       dim3(rc_blocks<M>(a.ny, a.nz, a.kr_max, a.kr_nb), a.batch ? a.nbatch : 1),
                       dim3(RC_NT), 0, s, a);
    return (int)hipGetLastError();
}

#define PK_CASE_RCB(N) case N: return rc_blocks<N>(ny, nz, kr_max, kr_nb);
#define PK_CASE_RC(N) case N: return run_rc<N>(a, s);

int residual_check_blocks(int nx, int ny, int nz, int kr_max, int kr_nb)
{
    switch (nx / 2) { PK_X_LENGTHS(PK_CASE_RCB) default: return -1; }
}

int x_res_slots(int nx, int xw, int p32) { return x_res_slots_f32(nx, xw, p32); }

template <int M> static int rc_slots()
{
    static int cache[64] = {0};
    int dev = 0;
    (void)hipGetDevice(&dev);
    int &r = cache[dev & 63];
    if (r == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_residual_check<M>, RC_NT, 0) !=
                hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || cus < 1) {
            (void)hipGetLastError();
            return -1;
        }
        r = per_cu * cus;
    }
    return r;
}
#define PK_CASE_RCS(N) case N: return rc_slots<N>();

int residual_check_slots(int nx)
{
    switch (nx / 2) { PK_X_LENGTHS(PK_CASE_RCS) default: return -1; }
}

int launch_residual_check(const XFwdArgs &a, int *nblocks_out, hipStream_t s)
{
    if (nblocks_out) *nblocks_out = residual_check_blocks(a.nx, a.ny, a.nz, a.kr_max, a.kr_nb);
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_RC) default: return -1; }
}

// Work list of residual checks of problems of different shapes (class: the
// half row length M; periodic and wall boxes alike)
#define PK_RL_LENGTHS(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

__global__ __launch_bounds__(RC_NT) void k_rc_list(ListArgs<XFwdArgs>)
{
    extern __shared__ __align__(16) char s_dyn[];
    const PK_KARG ListArgs<XFwdArgs> *L = list_args<XFwdArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const XFwdArgs arg = L->a[g];
    switch (L->cls[g]) {
#define PK_RL_CASE(N) case N: RCBody<N>::run(arg, vb, s_dyn); break;
        PK_RL_LENGTHS(PK_RL_CASE)
#undef PK_RL_CASE
    default: break;
    }
}

int launch_residual_check_list(const XFwdArgs *a, int n, hipStream_t s)
{
    ListArgs<XFwdArgs> L{};
    size_t lds = 0;
    int total = 0;
    auto flush = [&]() -> int {
        if (L.nseg == 0) return 0;
        L.start[L.nseg] = total;
        hipLaunchKernelGGL(k_rc_list, dim3(total), dim3(RC_NT), lds, s, L);
        L.nseg = 0;
        total = 0;
        lds = 0;
        return (int)hipGetLastError();
    };
    for (int i = 0; i < n; ++i) {
        size_t b = 0;
        switch (a[i].nx / 2) {
#define PK_RL_INFO(N) case N: b = RCBody<N>::LDS_BYTES; break;
            PK_RL_LENGTHS(PK_RL_INFO)
#undef PK_RL_INFO
        default: break;
        }
        if (b == 0) {
            const int e = launch_residual_check(a[i], nullptr, s);
            if (e) return e;
            continue;
        }
        const int gx = residual_check_blocks(a[i].nx, a[i].ny, a[i].nz, a[i].kr_max, a[i].kr_nb);
        const int g = L.nseg++;
        L.start[g] = total;
        L.gx[g] = gx;
        L.cls[g] = a[i].nx / 2;
        L.nt[g] = RC_NT;
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

// Sums of the partial records of several groups: one workgroup per problem
// of every segment (the problem's records, its scalars and control record
// from its ProbPtrs entry)
__global__ __launch_bounds__(1024) void k_sum_list(ListArgs<SumSeg>, double rtol, int max_refine)
{
    __shared__ double sh[3][1024];
    const PK_KARG ListArgs<SumSeg> *L = list_args<SumSeg>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const SumSeg sg = L->a[g];
    const ProbPtrs *batch = sg.batch;
    const int i = vb.y;
    if (gated_off(batch, sg.gate, i)) return;
    const double *in = batch[i].partials;
    double *out = batch[i].scal + sg.out_off;
    int n = sg.n;
    if (sg.mode == 2 && batch[i].ctrl[C_CHECK]) n = sg.n_check;
    double s0, s1, s2;
    sum_records(in, n, sh, s0, s1, s2);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
        if (sg.mode == 1) ctrl_open(batch[i].ctrl, batch[i].scal);
        if (sg.mode == 2) ctrl_decide(batch[i].ctrl, batch[i].scal, rtol, max_refine);
    }
}

int launch_sum_partials_list(const SumSeg *segs, int nseg, double rtol, int max_refine,
                             hipStream_t s)
{
    ListArgs<SumSeg> L{};
    int total = 0;
    for (int i = 0; i < nseg; ++i) {
        if (!segs[i].batch || segs[i].nbatch < 1) continue;
        if (L.nseg == LIST_MAX_SEG) {
            L.start[L.nseg] = total;
            hipLaunchKernelGGL(k_sum_list, dim3(total), dim3(1024), 0, s, L, rtol, max_refine);
            const int e = (int)hipGetLastError();
            if (e) return e;
            L.nseg = 0;
            total = 0;
        }
        const int g = L.nseg++;
        L.start[g] = total;
        L.gx[g] = 1;
        L.cls[g] = 0;
        L.nt[g] = 1024;
        L.a[g] = segs[i];
        total += segs[i].nbatch;
    }
    if (L.nseg == 0) return 0;
    L.start[L.nseg] = total;
    hipLaunchKernelGGL(k_sum_list, dim3(total), dim3(1024), 0, s, L, rtol, max_refine);
    return (int)hipGetLastError();
}

// Velocity correction and pressure update of the projection step
// (CorrMarch of stencil.hpp): streams psi once (plus halos) and u, v, w and p
// once each way.  512 threads per plane tile of about 1024 pairs (two each):
// at nx = 512 98 VGPRs and four waves per SIMD, against 182 and two with 256.
constexpr int CO_NT = 512;

// about 1024 pairs per plane tile: each element holds six double2 (psi at
// k and k+1, u, v, w, p) in registers
template <int M> constexpr int corr_rows() { return march_rows(M, 1024); }

template <int M>
__global__ __launch_bounds__(CO_NT) void k_correct(CorrArgs a)
{
    constexpr int TJ = corr_rows<M>();
    using Mar = CorrMarch<M, TJ, CO_NT>;
    __shared__ double2 s_tile[TJ + 1][M];
    const int njb = march_jblocks(a.ny, TJ);
    const int bid = xcd_order(blockIdx.x, gridDim.x);
    const int jb = bid % njb, kb = bid / njb;
    const int kr = march_planes(a.ny, a.nz, TJ, a.kr_max);
    const int k0 = kb * kr;
    const int k1 = k0 + kr < a.nz ? k0 + kr : a.nz;
    Mar m;
    m.psi = gbl(a.psi);
    m.u = gbl(a.u);
    m.v = gbl(a.v);
    m.w = gbl(a.w);
    m.p = a.p ? gbl(a.p) : nullptr;
    m.bx = a.bx;
    m.by = a.by;
    m.bz = a.bz;
    m.xwall = a.xwall != 0;
    m.ywall = a.ywall != 0;
    m.tile = s_tile;
    m.setup(jb, a.ny, a.nz, a.bc_z);
    m.start(k0);
    for (int k = k0; k < k1; ++k) {
        if (k > k0) __syncthreads();
        m.step(k);
    }
}

template <int M> static int run_correct(const CorrArgs &a, hipStream_t s)
{
    constexpr int TJ = corr_rows<M>();
    const int nb = march_jblocks(a.ny, TJ) * march_kblocks(a.ny, a.nz, TJ, a.kr_max);
    hipLaunchKernelGGL(k_correct<M>, dim3(nb), dim3(CO_NT), 0, s, a);
    return (int)hipGetLastError();
}

#define PK_CASE_CO(N) case N: return run_correct<N>(a, s);

// p = p32 widened to FP64 (the refinement's first iterate as the solution of
// a problem that stopped before any correction), n points
__global__ __launch_bounds__(256) void k_widen(const float *src, double *dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = (double)src[i];
}

int launch_widen(const float *src, double *dst, size_t n, hipStream_t s)
{
    if (!src || !dst || n == 0) return (int)hipErrorInvalidValue;
    const size_t want = (n + 255) / 256;
    const int nb = (int)(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_widen, dim3(nb), dim3(256), 0, s, src, dst, n);
    return (int)hipGetLastError();
}

// zero n 4-byte words (control records and scalars of a plan whose state
// must start cleared; a kernel rather than a memset so the clear also
// behaves inside a captured graph)
__global__ __launch_bounds__(256) void k_zero_words(unsigned *dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = 0u;
}

int launch_zero(void *dst, size_t bytes, hipStream_t s)
{
    if (!dst || bytes % 4) return (int)hipErrorInvalidValue;
    const size_t n = bytes / 4;
    if (n == 0) return 0;
    const size_t want = (n + 255) / 256;
    const int nb = (int)(want < 1024 ? want : 1024);
    hipLaunchKernelGGL(k_zero_words, dim3(nb), dim3(256), 0, s, (unsigned *)dst, n);
    return (int)hipGetLastError();
}

int launch_correct(const CorrArgs &a, hipStream_t s)
{
    switch (a.nx / 2) { PK_X_LENGTHS(PK_CASE_CO) default: return -1; }
}

}  // namespace pk
