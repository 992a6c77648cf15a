// k_misc.hip -- precision dispatch of the pass launchers and the
// deterministic FP64 reduction of per-workgroup partial sums (residual and
// right-hand-side norms of the iterative refinement).
#include "common.hpp"
#include "lengths.hpp"

namespace pk {

int launch_x_fwd_f32(const XFwdArgs &, hipStream_t);
int launch_x_fwd_f64(const XFwdArgs &, hipStream_t);
int launch_x_inv_f32(const XInvArgs &, hipStream_t);
int launch_x_inv_f64(const XInvArgs &, hipStream_t);
int launch_y_f32(const YArgs &, hipStream_t);
int launch_y_f64(const YArgs &, hipStream_t);
int launch_z_walls_f32(const ZArgs &, hipStream_t);
int launch_z_walls_f64(const ZArgs &, hipStream_t);
int launch_z_periodic_f32(const ZArgs &, hipStream_t);
int launch_z_periodic_f64(const ZArgs &, hipStream_t);
int x_fwd_blocks_f32(int, int, int);
int x_fwd_blocks_f64(int, int, int);

int launch_x_fwd(int prec, const XFwdArgs &a, int *nblocks_out, hipStream_t s)
{
    if (nblocks_out) *nblocks_out = x_fwd_blocks(prec, a.nx, a.ny, a.nz);
    return prec == P_F32 ? launch_x_fwd_f32(a, s) : launch_x_fwd_f64(a, s);
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
int x_fwd_blocks(int prec, int nx, int ny, int nz)
{
    return prec == P_F32 ? x_fwd_blocks_f32(nx, ny, nz) : x_fwd_blocks_f64(nx, ny, nz);
}

#define PK_IS(N) case N: return true;
bool fft_length_supported(int n)
{
    switch (n) { PK_LENGTHS(PK_IS) default: return false; }
}

// One workgroup per problem; thread t sums the 4-wide partial records t,
// t+1024, ... in a fixed order, then a fixed-shape tree finishes: bitwise
// reproducible for a given n.
__global__ __launch_bounds__(1024) void k_sum_partials(const double *in, int n, double *out,
                                                       const ProbPtrs *batch, int out_off)
{
    __shared__ double sh[3][1024];
    if (batch) {
        in = batch[blockIdx.x].partials;
        out = batch[blockIdx.x].scal + out_off;
    }
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = t; i < n; i += 1024) {
        const double4 v = *(const double4 *)(in + 4 * (size_t)i);
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
    if (t < 3) out[t] = sh[t][0];
}

int launch_sum_partials(const double *in, int n, double *out, const ProbPtrs *batch,
                        int nbatch, int out_off, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(batch ? nbatch : 1), dim3(1024), 0, s, in, n, out,
                       batch, out_off);
    return (int)hipGetLastError();
}

// Residual of the discrete equation, r = (f - mean f) - L p, in FP64 (the
// 7-point operator of the marker-and-cell grid: periodic x and y, z periodic
// or mirrored ghost at the walls).  Streams f and p once; a workgroup owns
// RB consecutive grid rows and writes three partial sums: sum r^2,
// sum (f - mean f)^2, sum p.
constexpr int RC_ROWS = 4;
constexpr int RC_THREADS = 256;

__device__ __forceinline__ void block_sum3_rc(double &a, double &b, double &c, double *sh)
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
        a = b = c = 0.0;
        for (int w = 0; w < RC_THREADS / 64; ++w) {
            a += sh[3 * w];
            b += sh[3 * w + 1];
            c += sh[3 * w + 2];
        }
    }
}

__global__ __launch_bounds__(RC_THREADS) void k_residual_check(XFwdArgs a0)
{
    __shared__ double s_red[3 * (RC_THREADS / 64)];
    XFwdArgs a = a0;
    if (a.batch) {
        const ProbPtrs &q = a.batch[blockIdx.y];
        a.f = q.f;
        a.p = q.p;
        a.partials = q.partials;
        a.sum_f = q.scal + 1;
    }
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int half = nx / 2;
    const int nrows = ny * nz;
    const int row0 = block_order(blockIdx.x, gridDim.x, a.reverse) * RC_ROWS;
    const double mu = a.sum_f ? (*a.sum_f) * a.inv_n : 0.0;
    const size_t plane = (size_t)ny * nx;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (int u = threadIdx.x; u < RC_ROWS * half; u += RC_THREADS) {
        const int row = row0 + u / half;
        const int n = u % half;
        if (row >= nrows) continue;
        const int j = row % ny, k = row / ny;
        const size_t roff = (size_t)row * nx;
        const double2 fv = *(const double2 *)(a.f + roff + 2 * n);
        const double *pr = a.p + roff;
        const double2 pc = *(const double2 *)(pr + 2 * n);
        const double pl = pr[(2 * n + nx - 1) % nx];
        const double pq = pr[(2 * n + 2) % nx];
        const int jm = (j == 0) ? ny - 1 : j - 1;
        const int jp = (j == ny - 1) ? 0 : j + 1;
        int km, kp;
        if (a.bc_z == 0) {
            km = (k == 0) ? nz - 1 : k - 1;
            kp = (k == nz - 1) ? 0 : k + 1;
        } else {
            km = (k == 0) ? 0 : k - 1;
            kp = (k == nz - 1) ? k : k + 1;
        }
        const double2 ps = *(const double2 *)(a.p + (size_t)k * plane + (size_t)jm * nx + 2 * n);
        const double2 pn = *(const double2 *)(a.p + (size_t)k * plane + (size_t)jp * nx + 2 * n);
        const double2 pd = *(const double2 *)(a.p + (size_t)km * plane + (size_t)j * nx + 2 * n);
        const double2 pu = *(const double2 *)(a.p + (size_t)kp * plane + (size_t)j * nx + 2 * n);
        const double l0 = a.ax * (pc.y - 2.0 * pc.x + pl) + a.ay * (pn.x - 2.0 * pc.x + ps.x) +
                          a.az * (pu.x - 2.0 * pc.x + pd.x);
        const double l1 = a.ax * (pq - 2.0 * pc.y + pc.x) + a.ay * (pn.y - 2.0 * pc.y + ps.y) +
                          a.az * (pu.y - 2.0 * pc.y + pd.y);
        const double f0 = fv.x - mu, f1 = fv.y - mu;
        const double r0 = f0 - l0, r1 = f1 - l1;
        acc0 += r0 * r0 + r1 * r1;
        acc1 += f0 * f0 + f1 * f1;
        acc2 += pc.x + pc.y;
    }
    block_sum3_rc(acc0, acc1, acc2, s_red);
    if (threadIdx.x == 0) {
        a.partials[4 * blockIdx.x] = acc0;
        a.partials[4 * blockIdx.x + 1] = acc1;
        a.partials[4 * blockIdx.x + 2] = acc2;
    }
}

int residual_check_blocks(int ny, int nz) { return (ny * nz + RC_ROWS - 1) / RC_ROWS; }

int launch_residual_check(const XFwdArgs &a, int *nblocks_out, hipStream_t s)
{
    const int nb = residual_check_blocks(a.ny, a.nz);
    if (nblocks_out) *nblocks_out = nb;
    hipLaunchKernelGGL(k_residual_check, dim3(nb, a.batch ? a.nbatch : 1), dim3(RC_THREADS), 0,
                       s, a);
    return (int)hipGetLastError();
}

}  // namespace pk
