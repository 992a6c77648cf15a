// common.hpp -- types and launcher declarations shared by the host plan code
// and the HIP kernels of the FFT-based Poisson solver (FluTAS, Section 3.3.1).
//
// Data layout in HBM
//   real fields  f, p : double, (nz, ny, nx), x fastest.
//   spectrum S        : complex<R>, (nz, ny, M) with M = nx/2, x-wavenumber
//                       fastest.  Column m = 0 packs the two real x-modes:
//                       S[.,.,0] = X(0) + i X(M) (DC and Nyquist of the real
//                       transform along x).  In FP64 mode S aliases the
//                       solution array (same byte size); in FP32 modes it is a
//                       separate workspace of 4 bytes per grid point.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace pk {

template <typename R>
struct Cx {
    R re, im;
};

// Loads and stores of device fields through the global address space.
// Pointers that reach a kernel through memory (the per-problem pointer table
// of batched launches) or through structs are generic to the compiler, which
// then emits flat instructions; flat loads also count against the LDS wait
// counter, so every LDS wait of an FFT or stencil tile would also wait for
// the outstanding HBM loads.  All fields live in device memory.
// The cast has to be applied to the base pointer, before any offset
// arithmetic (a cast of a derived generic pointer is folded back into a
// flat access), hence gbl() at the point where a kernel obtains a pointer.
// (device compilation pass only; the host pass parses the same templates
// with plain pointers)
#if defined(__HIP_DEVICE_COMPILE__)
#define PK_GLOBAL __attribute__((address_space(1)))
#else
#define PK_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ PK_GLOBAL T *gbl(T *p)
{
    return (PK_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const PK_GLOBAL T *gbl(const T *p)
{
    return (const PK_GLOBAL T *)p;
}
// store of a complex value through a global pointer (member-wise: the
// implicit assignment operator does not take an address-space-qualified
// object; the two stores are merged into one vector store)
template <typename R>
__device__ __forceinline__ void put(PK_GLOBAL Cx<R> *p, Cx<R> v)
{
    p->re = v.re;
    p->im = v.im;
}

// Streaming (non-temporal) access to pairs of doubles that a kernel touches
// once and no later pass reads soon: the lines are marked for early eviction
// instead of displacing data the next pass still finds in the caches.
// Measured on MI355X: +7 % for the read-modify-write velocity correction.
typedef double pk_d2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const PK_GLOBAL double *p)
{
    const pk_d2v v = __builtin_nontemporal_load((const PK_GLOBAL pk_d2v *)p);
    return double2{v.x, v.y};
}
__device__ __forceinline__ void st_stream(PK_GLOBAL double *p, double2 a)
{
    const pk_d2v v = {a.x, a.y};
    __builtin_nontemporal_store(v, (PK_GLOBAL pk_d2v *)p);
}
// the same for a pair held in FP32 (widened / narrowed exactly by callers
// whose values are FP32 numbers)
typedef float pk_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const PK_GLOBAL float *p)
{
    const pk_f2v v = __builtin_nontemporal_load((const PK_GLOBAL pk_f2v *)p);
    return double2{(double)v.x, (double)v.y};
}
__device__ __forceinline__ void st_stream(PK_GLOBAL float *p, double2 a)
{
    const pk_f2v v = {(float)a.x, (float)a.y};
    __builtin_nontemporal_store(v, (PK_GLOBAL pk_f2v *)p);
}

enum Prec { P_F64 = 0, P_F32 = 1 };

// Block order.  A pass whose input was just written by the previous pass
// starts on the data that pass wrote last when `reverse` is set: the most
// recently written lines are the ones still held by the 256 MB last-level
// (Infinity) cache, so reading them first turns part of the pass's HBM reads
// into cache hits instead of evicting them before use.
__device__ __forceinline__ int block_order(int bid, int nblocks, int reverse)
{
    return reverse ? nblocks - 1 - bid : bid;
}

// Workgroup i of a launch starts on accelerator die (XCD) i % 8, and each
// die has its own L2.  xcd_order maps the launch index to a logical block
// index such that every die walks a contiguous run of logical blocks: blocks
// that share halo rows run on the same die at about the same time and share
// its L2.  A bijection on [0, nblocks).
__device__ __forceinline__ int xcd_order(int bid, int nblocks)
{
    constexpr int X = 8;
    const int q = nblocks / X, rem = nblocks % X;
    const int x = bid % X, slot = bid / X;
    return x * q + (x < rem ? x : rem) + slot;
}

// Per-problem pointers of a batched launch: problems of one shape share a
// launch and blockIdx.y selects the entry.  A null `batch` pointer in the
// argument structs below means a single-problem launch using their own
// pointers.
struct ProbPtrs {
    const double *f;   // right-hand side
    double *p;         // solution
    void *S;           // spectrum
    double *partials;  // per-workgroup partial sums of the x pass
    double *scal;      // 8 FP64 scalars: [0] mean (z pass), [1] sum f, [2] sum r^2,
                       // [3] sum (f - mean)^2, [4] sum p, [5] relative residual,
                       // [6] previous relative residual, [7] first relative residual
    int *ctrl;         // refinement control record (device-side loop), CtrlSlot
    float *p32;        // refinement: the first iterate, exactly, in FP32 (or null)
};

// Device-side control of the refinement loop: one record of NCTRL ints per
// problem.  Passes of the loop carry a `gate` slot (0: none) and a workgroup
// of problem i returns at once when ctrl[gate] of problem i is zero, so a
// fixed launch sequence (a captured graph) serves problems that converge
// after different numbers of corrections.
enum CtrlSlot {
    C_STATE = 0,    // 1 while the problem is running
    C_FULL = 1,     // next residual: full residual pass (with transform)
    C_CHECK = 2,    // next residual: check only
    C_EVAL = 3,     // a residual is evaluated in this segment (C_FULL or C_CHECK)
    C_FIX = 4,      // a check failed: transform the residual before correcting
    C_CORRECT = 5,  // run the correction passes
    C_CORR = 6,     // corrections applied so far
    C_STATUS = 7,   // final status (poisson error code)
    C_COPY = 8,     // done before any correction: the solution is the first iterate
    NCTRL = 9
};

__device__ __forceinline__ bool gated_off(const ProbPtrs *batch, int gate, int i)
{
    return gate != 0 && batch != nullptr && batch[i].ctrl[gate] == 0;
}

// Arguments of the forward real-to-complex pass along x (optionally with the
// FP64 residual r = (f - mu) - L p evaluated on the fly as its input).
struct XFwdArgs {
    const ProbPtrs *batch;  // batched launch (or null)
    int nbatch;             // gridDim.y
    const double *f;        // (nz, ny, nx)
    const double *p;        // residual mode only: current solution
    void *S;                // complex<R> spectrum, row pitch M
    const void *tw;         // complex<R> table exp(-2 pi i t/nx), t in [0, nx)
    double *partials;       // per-workgroup FP64 sums (nullable)
    int nx, ny, nz;
    int bc_z;               // 0 periodic, 1 Neumann walls, 2 Dirichlet walls
    int bc_y;               // the same along y (residual marches)
    int bc_x;               // the same along x: walls take cosine / sine expansions
    const void *tw4x;       // walls along x: exp(-i pi k/(2 nx)), k in [0, nx)
    double ax, ay, az;      // 1/dx^2, 1/dy^2, 1/dz^2
    const double *sum_f;    // residual mode: device sum of f (mean = sum_f * inv_n)
    double inv_n;           // 1/(nx ny nz)
    int residual;           // 1: input is the residual; 2: the divergence of (u, v, w)
    int reverse;            // walk the row blocks from the end (see block_order)
    int gate;               // control slot gating this launch (0: none)
    int kr_max;             // residual passes: z-planes per workgroup (0: default)
    int kr_nb;              // residual passes: problems of the group (march_planes)
    int p_in32;             // residual pass: p is the FP32 first iterate (p32 / batch[i].p32)
    const float *p32;
    int regular;            // a Dirichlet wall: no null space, f keeps its mean
    // divergence input (residual == 2; one problem): f = cx Dx u + cy Dy v + cz Dz w
    const double *u, *v, *w;
    double cx, cy, cz;      // alpha/dx, alpha/dy, alpha/dz
    double *f_out;          // receives f in FP64 (nullable)
    // stretched z (null: uniform): hz[k] the thickness of plane k, weighting
    // the sums of f and p (volume-weighted means; inv_n is then
    // 1/(nx ny sum h)); zc[2k], zc[2k+1] the z coefficients of plane k in
    // the residual, (a_k, c_k)/h_k with a Dirichlet wall's 1/h_k^2 (its
    // ghost plane is the negated wall plane)
    const double *hz;
    const double *zc;
};

// Inverse complex-to-real pass along x: p = result (store) or p += result.
struct XInvArgs {
    const ProbPtrs *batch;
    int nbatch;
    const void *S;
    double *p;
    const void *tw;
    int nx, ny, nz;
    int accumulate;
    int reverse;
    const double *sum_p;    // accumulate mode: device sum of p (its mean is removed)
    double inv_n;           // 1/(nx ny nz)
    int gate;
    int regular;            // a Dirichlet wall: the mean of p is kept
    int bc_x;               // 0 periodic, 1 Neumann walls (cosines), 2 Dirichlet walls (sines)
    const void *tw4x;       // walls along x: exp(-i pi k/(2 nx)), k in [0, nx)
    // refinement with the first iterate kept in FP32: the plain pass writes
    // it to p32; the accumulating pass reads it from p32 and writes p (or,
    // for a problem whose control record says C_COPY, only widens p32 to p)
    int p_in32;
    float *p32;
};

// Strided complex pass along y, in place on S.
struct YArgs {
    const ProbPtrs *batch;
    int nbatch;
    void *S;
    const void *tw;         // exp(-2 pi i t/ny), t in [0, ny)
    int M, ny, nz;
    int inverse;
    int reverse;
    int gate;
    int variant;            // tile variant (see YCfg)
    int bc;                 // 0 periodic (FFT), 1 Neumann walls (cosines), 2 Dirichlet (sines)
    const void *tw4;        // walls: exp(-i pi k/(2 ny)), k in [0, ny)
};

// z solve, walls (tridiagonal per (m, ky)) or periodic (transform along z).
struct ZArgs {
    const ProbPtrs *batch;
    int nbatch;
    void *S;
    const void *tw;         // periodic: exp(-2 pi i t/nz)
    const double *lamx;     // lambda_x(m), m in [0, M]
    const double *lamy;     // lambda_y(ky), ky in [0, ny)
    const double *lamz;     // periodic: lambda_z(kz), kz in [0, nz)
    double *zero_mean_out;  // receives mean(f) from the zero-wavenumber column
    int M, ny, nz;
    int nx;
    double dz2;             // dz^2
    double inv_nxny;        // 1/(nx ny)
    double inv_ntot;        // 1/(nx ny nz)
    int reverse;
    int variant;            // tile variant (0 = default; see the launchers)
    int gate;
    int dirichlet_z;        // walls with zero value (ghost = -wall cell) instead of zero gradient
    int regular;            // no null space (a Dirichlet wall on some axis): no zero mode
    int ywall;              // walls along y: the m = 0 column holds A + iB with real y-modes
    int xwall;              // walls along x: every column m holds the real x-modes 2m, 2m+1
    int periodic_z;         // 1: periodic z (transform), 0: walls (tridiagonal solve)
    // stretched z (walls; cells of thickness h_k): 8 doubles per row k,
    // {a_k, c_k, h_k, D_k, d_k+1/2, sum_{j<k} h_j, 0, 0} with a_k, c_k the
    // conductances 1/d of the faces below and above (0 at a wall), D_k the
    // Dirichlet wall term 2/h_k, d_k+1/2 the distance of the centres k, k+1;
    // rows from nz on are padding {0, 0, 0, 1, 0, sum h, 0, 0}.  Null: uniform.
    const double *zrow;
    double hsum;            // sum of the thicknesses
};

// ---------------------------------------------------------------------------
// Work lists: one launch serving problems of different shapes.  The blocks of
// a list launch are dealt out to segments, one per shape group; segment g
// covers blocks [start[g], start[g+1]) and serves nbatch problems of one
// shape with gx blocks each: its relative block b is block (b % gx, b / gx)
// of that group's own launch.  The body that runs is picked by the segment's
// class (a transform length and its compile-time variant); it uses the first
// nt threads of the workgroup (the others leave at once) and carves its LDS
// from the launch's dynamic LDS.
// ---------------------------------------------------------------------------
struct VBlock {
    int x, y, gx;  // block within the group's launch, problem, blocks per problem
};

constexpr int LIST_MAX_SEG = 8;

template <class A>
struct ListArgs {
    int nseg;
    int start[LIST_MAX_SEG + 1];
    int gx[LIST_MAX_SEG];
    int cls[LIST_MAX_SEG];   // class of the segment's body
    int nt[LIST_MAX_SEG];    // threads its body uses
    int aux[LIST_MAX_SEG];   // per-class launch parameters (chunks, special blocks)
    int aux2[LIST_MAX_SEG];
    A a[LIST_MAX_SEG];
};

// The list kernels take one argument, the ListArgs, and read it through the
// kernel argument segment's address (constant address space: scalar loads
// at any segment index; an indexed copy of the by-value argument would be
// placed in scratch memory).
#if defined(__HIP_DEVICE_COMPILE__)
#define PK_KARG __attribute__((address_space(4)))
#else
#define PK_KARG
#endif
template <class A>
__device__ __forceinline__ const PK_KARG ListArgs<A> *list_args()
{
    return (const PK_KARG ListArgs<A> *)__builtin_amdgcn_kernarg_segment_ptr();
}

// Segment and virtual block of this workgroup; false when the thread is
// beyond the body's threads (it has nothing to do).  The bodies check their
// problem's gate themselves.
template <class A>
__device__ __forceinline__ bool list_find(const PK_KARG ListArgs<A> *L, int &g, VBlock &vb)
{
    const int b = (int)blockIdx.x;
    int i = 0;
    while (i + 1 < L->nseg && b >= L->start[i + 1]) ++i;
    g = i;
    const int local = b - L->start[i];
    const int gx = L->gx[i];
    vb.y = local / gx;
    vb.x = local - vb.y * gx;
    vb.gx = gx;
    return (int)threadIdx.x < L->nt[i];
}

// Launchers (return 0 on success, a hipError_t value otherwise).  The forward
// x pass reports the workgroups it launched (the partial sums it wrote).
int launch_x_fwd(int prec, const XFwdArgs &a, int *nblocks_out, hipStream_t s);
int launch_x_inv(int prec, const XInvArgs &a, hipStream_t s);
int launch_y(int prec, const YArgs &a, hipStream_t s);
int launch_z_walls(int prec, const ZArgs &a, hipStream_t s);
int launch_z_periodic(int prec, const ZArgs &a, hipStream_t s);
// number of workgroups the forward x pass uses (size of its partials array);
// `residual` selects the residual pass of the refinement
int x_fwd_blocks(int prec, int nx, int ny, int nz, int residual, int kr_max, int kr_nb = 1);
// Deterministic FP64 sums of the x pass's partials: `n` workgroups with three
// sums each (stride 4), written to out[0..3).  Batched: one workgroup per
// problem, partials and scal taken from batch[i], written to scal + out_off.
// Batched launches of the device-side loop also take the control step of
// each problem (CtrlSlot records): mode 1 opens the record, mode 2 decides
// after a residual evaluation (rtol, max_refine); in mode 2, n counts the
// records of the residual pass with transform and n_check those of the
// residual check (the problem's C_CHECK flag tells which one ran).
int launch_sum_partials(const double *in, int n, double *out, const ProbPtrs *batch,
                        int nbatch, int out_off, hipStream_t s, int gate = 0, int mode = 0,
                        double rtol = 0.0, int max_refine = 0, int n_check = 0);
// FP64 residual r = (f - mean f) - L p alone (no transform, no spectrum
// write): per-workgroup sums of r^2, (f - mean f)^2 and p into `partials`
// (same layout as the forward x pass), for a convergence check.
int launch_residual_check(const XFwdArgs &a, int *nblocks_out, hipStream_t s);
int residual_check_blocks(int nx, int ny, int nz, int kr_max, int kr_nb = 1);
// workgroups of the residual pass with transform (rows of nx points, walls
// along x or not, p in FP32 or FP64) and of the residual check that the
// current device holds at once (occupancy x compute units); -1 if unknown
int x_res_slots(int nx, int xw, int p32);
int residual_check_slots(int nx);
// dst[i] = (double)src[i], i < n (device arrays)
int launch_widen(const float *src, double *dst, size_t n, hipStream_t s);
// clear `bytes` (a multiple of 4) at dst with a kernel
int launch_zero(void *dst, size_t bytes, hipStream_t s);

// Work-list launchers: n argument records of one pass kind, one per shape
// group (batched records), served by as few launches as possible (one per
// LIST_MAX_SEG groups); a group outside the list kernels' classes gets its
// own launch of the per-group launcher.  x passes: all records plain
// (residual = 0, periodic x) or all residual; y: all forward or all inverse;
// z: walls and periodic records mixed.
int launch_y_list(int prec, const YArgs *a, int n, hipStream_t s);
int launch_z_list(int prec, const ZArgs *a, int n, hipStream_t s);
int launch_x_fwd_list(int prec, const XFwdArgs *a, int n, hipStream_t s);
int launch_x_inv_list(int prec, const XInvArgs *a, int n, hipStream_t s);
int launch_residual_check_list(const XFwdArgs *a, int n, hipStream_t s);
// workgroups of a group's forward x pass in a list launch (its partial
// records): plain passes take one tile of rows per workgroup
int x_fwd_list_blocks(int prec, const XFwdArgs &a);
// sum of the partial records of several groups (batched records), one
// workgroup per problem: n records per problem of group i, or n_check when
// the problem's control record says a residual check ran (mode 2)
struct SumSeg {
    const ProbPtrs *batch;
    int nbatch;
    int n, n_check;
    int out_off, gate, mode;
};
int launch_sum_partials_list(const SumSeg *segs, int nseg, double rtol, int max_refine,
                             hipStream_t s);

// Velocity correction and pressure update of the projection step:
// u -= bx Dx+ psi, v -= by Dy+ psi, w -= bz Dz+ psi (not on a top wall),
// p += psi when p is not null; one problem, arrays (nz, ny, nx).
struct CorrArgs {
    const double *psi;
    double *u, *v, *w, *p;
    int nx, ny, nz, bc_z;
    double bx, by, bz;      // beta/dx, beta/dy, beta/dz
    int kr_max;             // z-planes per workgroup (0: default)
    int xwall, ywall;       // solid walls along x / y (wall faces left as they are)
};
int launch_correct(const CorrArgs &a, hipStream_t s);

// lengths supported by the transform kernels
bool fft_length_supported(int n);

}  // namespace pk
