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

// One workgroup per problem; thread t sums entries t, t+256, ... of each of
// the three interleaved streams (stride 4) in a fixed order, then a
// fixed-shape tree finishes: bitwise reproducible for a given n.
__global__ __launch_bounds__(256) void k_sum_partials(const double *in, int n, double *out,
                                                      const ProbPtrs *batch, int out_off)
{
    __shared__ double sh[256];
    if (batch) {
        in = batch[blockIdx.x].partials;
        out = batch[blockIdx.x].scal + out_off;
    }
    constexpr int nsums = 3, stride = 4;
    for (int s = 0; s < nsums; ++s) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += 256) acc += in[(size_t)i * stride + s];
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[s] = sh[0];
        __syncthreads();
    }
}

int launch_sum_partials(const double *in, int n, double *out, const ProbPtrs *batch,
                        int nbatch, int out_off, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(batch ? nbatch : 1), dim3(256), 0, s, in, n, out,
                       batch, out_off);
    return (int)hipGetLastError();
}

}  // namespace pk
