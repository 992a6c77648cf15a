// k_xlist.hip -- work lists of the x passes (steps 1 and 9 of the solve
// sequence in FluTAS Section 3.3.1, and the residual pass of the iterative
// refinement): the forward, residual and inverse x passes of problems of
// different shapes in one launch each.  Segment classes are the half row
// length M (and the variant flags); the bodies are those of k_xpass.hip, the
// plain forward pass taking one tile of rows per workgroup (the per-group
// launch is persistent).  Periodic x only: groups with walls along x keep
// their own launches.
//
// Compiled once per precision with PK_REAL = float or double.
#define PK_X_LIST_TU
#include "k_xpass.hip"

namespace pk {
namespace PK_NS {

// Plain forward pass, one tile of NB rows: rows of f transformed into the
// half spectrum, the FP64 sum of f into the workgroup's partial record.
template <int M> struct XFPlainBody {
    using C = XCfg<M>;
    static constexpr int NB = C::NB, NT = C::NT, NX = 2 * M;
    using Tile = LdsTile<R, M, NB, false, 0>;
    static constexpr size_t TILE0 = sizeof(Cx<R>) * Tile::elems;
    static constexpr size_t RED = sizeof(double) * 3 * (NT / 64);
    static constexpr size_t TILE_B = ((TILE0 > RED ? TILE0 : RED) + 15) / 16 * 16;
    static constexpr size_t LDS_BYTES = TILE_B + sizeof(Cx<R>) * NX;

    static __device__ __forceinline__ void run(const XFwdArgs &a0, VBlock vb, char *lds)
    {
        if (gated_off(a0.batch, a0.gate, vb.y)) return;
        XFwdArgs a = a0;
        if (a.batch) {
            const ProbPtrs &q = a.batch[vb.y];
            a.f = q.f;
            a.S = q.S;
            if (a.partials) a.partials = q.partials;
        }
        Cx<R> *s_tile = (Cx<R> *)lds;
        Cx<R> *s_tw = (Cx<R> *)(lds + TILE_B);
        const int nrows = a.ny * a.nz;
        load_table(s_tw, (const Cx<R> *)a.tw, NX, NT);
        __syncthreads();
        const int row0 = block_order(vb.x, vb.gx, a.reverse) * NB;
        const PK_GLOBAL double *gf = gbl(a.f);
        PK_GLOBAL Cx<R> *S = gbl((Cx<R> *)a.S);
        double acc0 = 0.0;
        auto gload = [&](int b, int n) -> Cx<R> {
            const int row = row0 + b;
            if (row >= nrows) return {R(0), R(0)};
            const double2 fv = ld_stream(gf + (size_t)row * NX + 2 * n);
            acc0 += (a.hz ? a.hz[row / a.ny] : 1.0) * (fv.x + fv.y);
            return {R(fv.x), R(fv.y)};
        };
        auto out = [&](int b) -> PK_GLOBAL Cx<R> * {
            const int row = row0 + b;
            return row < nrows ? S + (size_t)row * M : nullptr;
        };
        Tile tile{s_tile};
        x_forward<M, NB, NT, false, 0, false>(s_tw, gload, tile, out);
        if (a.partials) {
            double *s_red = (double *)s_tile;
            double z1 = 0.0, z2 = 0.0;
            __syncthreads();
            block_sum3(acc0, z1, z2, s_red, NT);
            if (threadIdx.x == 0) {
                a.partials[4 * vb.x] = acc0;
                a.partials[4 * vb.x + 1] = 0.0;
                a.partials[4 * vb.x + 2] = 0.0;
            }
        }
    }
};

constexpr int XL_NT = 256;
#define PK_XL_LENGTHS(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128)

__global__ __launch_bounds__(XL_NT) void k_xf_list(ListArgs<XFwdArgs>)
{
    extern __shared__ __align__(16) char s_dyn[];
    const PK_KARG ListArgs<XFwdArgs> *L = list_args<XFwdArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const XFwdArgs arg = L->a[g];
    switch (L->cls[g]) {
#define PK_XF_CASE(N)                                                                 \
    case N:                                                                           \
        if constexpr (XCfg<N>::NT <= XL_NT) XFPlainBody<N>::run(arg, vb, s_dyn);   \
        break;
        PK_XL_LENGTHS(PK_XF_CASE)
#undef PK_XF_CASE
    default: break;
    }
}

// residual pass: class 2 M + (p read from the FP32 first iterate)
__global__ __launch_bounds__(XR_NT) void k_xr_list(ListArgs<XFwdArgs>)
{
    extern __shared__ __align__(16) char s_dyn[];
    const PK_KARG ListArgs<XFwdArgs> *L = list_args<XFwdArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const XFwdArgs arg = L->a[g];
    switch (L->cls[g]) {
#define PK_XR_CASE(N)                                                          \
    case 2 * N: XRBody<N, false, false>::run(arg, vb, s_dyn); break;        \
    case 2 * N + 1:                                                            \
        if constexpr (sizeof(R) == 4) XRBody<N, false, true>::run(arg, vb, s_dyn); \
        break;
        PK_XL_LENGTHS(PK_XR_CASE)
#undef PK_XR_CASE
    default: break;
    }
}

// inverse pass: class 4 M + 2 accumulate + (FP32 first iterate)
__global__ __launch_bounds__(XL_NT) void k_xi_list(ListArgs<XInvArgs>)
{
    extern __shared__ __align__(16) char s_dyn[];
    const PK_KARG ListArgs<XInvArgs> *L = list_args<XInvArgs>();
    int g;
    VBlock vb;
    if (!list_find(L, g, vb)) return;
    const XInvArgs arg = L->a[g];
    switch (L->cls[g]) {
#define PK_XI_CASE(N)                                                                        \
    case 4 * N:                                                                              \
        if constexpr (XCfg<N>::NT <= XL_NT) XIBody<N, false, false, false>::run(arg, vb, s_dyn); \
        break;                                                                               \
    case 4 * N + 1:                                                                          \
        if constexpr (XCfg<N>::NT <= XL_NT && sizeof(R) == 4)                                \
            XIBody<N, false, false, true>::run(arg, vb, s_dyn);                           \
        break;                                                                               \
    case 4 * N + 2:                                                                          \
        if constexpr (XCfg<N>::NT <= XL_NT) XIBody<N, true, false, false>::run(arg, vb, s_dyn); \
        break;                                                                               \
    case 4 * N + 3:                                                                          \
        if constexpr (XCfg<N>::NT <= XL_NT && sizeof(R) == 4)                                \
            XIBody<N, true, false, true>::run(arg, vb, s_dyn);                            \
        break;
        PK_XL_LENGTHS(PK_XI_CASE)
#undef PK_XI_CASE
    default: break;
    }
}

// class information of the records (false: no list class, own launch)
static bool xf_list_class(const XFwdArgs &a, int &nt, int &gx, size_t &lds)
{
    if (a.bc_x != 0 || a.residual != 0) return false;
    switch (a.nx / 2) {
#define PK_XF_INFO(N)                                                 \
    case N: {                                                         \
        using B = XFPlainBody<N>;                                     \
        if (B::NT > XL_NT) return false;                              \
        nt = B::NT;                                                   \
        gx = (a.ny * a.nz + B::NB - 1) / B::NB;                       \
        lds = B::LDS_BYTES;                                           \
        return true;                                                  \
    }
        PK_XL_LENGTHS(PK_XF_INFO)
#undef PK_XF_INFO
    default: return false;
    }
}

static bool xr_list_class(const XFwdArgs &a, int &nt, int &gx, size_t &lds)
{
    if (a.bc_x != 0 || a.residual != 1) return false;
    if (a.p_in32 && sizeof(R) != 4) return false;
    switch (a.nx / 2) {
#define PK_XR_INFO(N)                                                                       \
    case N: {                                                                               \
        nt = XR_NT;                                                                         \
        gx = march_jblocks(a.ny, march_rows_res(N)) *                                       \
             march_kblocks(a.ny, a.nz, march_rows_res(N), a.kr_max, a.kr_nb);               \
        lds = a.p_in32 ? XRBody<N, false, true>::LDS_BYTES : XRBody<N, false, false>::LDS_BYTES; \
        return true;                                                                        \
    }
        PK_XL_LENGTHS(PK_XR_INFO)
#undef PK_XR_INFO
    default: return false;
    }
}

static bool xi_list_class(const XInvArgs &a, int &nt, int &gx, size_t &lds)
{
    if (a.bc_x != 0) return false;
    if (a.p_in32 && sizeof(R) != 4) return false;
    switch (a.nx / 2) {
#define PK_XI_INFO(N)                                                 \
    case N: {                                                         \
        using C = XCfg<N>;                                            \
        if (C::NT > XL_NT) return false;                              \
        nt = C::NT;                                                   \
        gx = (a.ny * a.nz + C::NB - 1) / C::NB;                       \
        lds = XIBody<N, false, false, false>::LDS_BYTES;              \
        return true;                                                  \
    }
        PK_XL_LENGTHS(PK_XI_INFO)
#undef PK_XI_INFO
    default: return false;
    }
}

// one launch per LIST_MAX_SEG supported records; the others on their own
template <class A, class Info, class Cls, class Launch, class Own>
static int run_list(const A *a, int n, hipStream_t s, Info info, Cls cls_of, Launch launch,
                    Own own)
{
    ListArgs<A> L{};
    size_t lds = 0;
    int total = 0;
    auto flush = [&]() -> int {
        if (L.nseg == 0) return 0;
        L.start[L.nseg] = total;
        const int e = launch(L, total, lds);
        L.nseg = 0;
        total = 0;
        lds = 0;
        return e;
    };
    for (int i = 0; i < n; ++i) {
        int nt = 0, gx = 0;
        size_t b = 0;
        if (!info(a[i], nt, gx, b)) {
            const int e = own(a[i]);
            if (e) return e;
            continue;
        }
        const int g = L.nseg++;
        L.start[g] = total;
        L.gx[g] = gx;
        L.cls[g] = cls_of(a[i]);
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

}  // namespace PK_NS
using namespace PK_NS;

int PK_SUFFIX(launch_x_fwd)(const XFwdArgs &a, hipStream_t s, int *nblocks_out);
int PK_SUFFIX(launch_x_inv)(const XInvArgs &a, hipStream_t s);

int PK_SUFFIX(launch_x_fwd_list)(const XFwdArgs *a, int n, hipStream_t s)
{
    if (n == 0) return 0;
    const bool res = a[0].residual == 1;
    for (int i = 0; i < n; ++i)
        if ((a[i].residual == 1) != res) return (int)hipErrorInvalidValue;
    auto own = [&](const XFwdArgs &r) { return PK_SUFFIX(launch_x_fwd)(r, s, nullptr); };
    if (res) {
        return run_list(
            a, n, s, [](const XFwdArgs &r, int &nt, int &gx, size_t &b) {
                return xr_list_class(r, nt, gx, b); },
            [](const XFwdArgs &r) { return r.nx + (r.p_in32 ? 1 : 0); },
            [&](const ListArgs<XFwdArgs> &L, int total, size_t lds) {
                hipLaunchKernelGGL(k_xr_list, dim3(total), dim3(XR_NT), lds, s, L);
                return (int)hipGetLastError();
            },
            own);
    }
    return run_list(
        a, n, s, [](const XFwdArgs &r, int &nt, int &gx, size_t &b) {
            return xf_list_class(r, nt, gx, b); },
        [](const XFwdArgs &r) { return r.nx / 2; },
        [&](const ListArgs<XFwdArgs> &L, int total, size_t lds) {
            hipLaunchKernelGGL(k_xf_list, dim3(total), dim3(XL_NT), lds, s, L);
            return (int)hipGetLastError();
        },
        own);
}

int PK_SUFFIX(launch_x_inv_list)(const XInvArgs *a, int n, hipStream_t s)
{
    return run_list(
        a, n, s, [](const XInvArgs &r, int &nt, int &gx, size_t &b) {
            return xi_list_class(r, nt, gx, b); },
        [](const XInvArgs &r) { return 2 * r.nx + 2 * (r.accumulate ? 1 : 0) + (r.p_in32 ? 1 : 0); },
        [&](const ListArgs<XInvArgs> &L, int total, size_t lds) {
            hipLaunchKernelGGL(k_xi_list, dim3(total), dim3(XL_NT), lds, s, L);
            return (int)hipGetLastError();
        },
        [&](const XInvArgs &r) { return PK_SUFFIX(launch_x_inv)(r, s); });
}

int PK_SUFFIX(x_fwd_grid)(const XFwdArgs &a);

// workgroups (partial records) of a record's forward pass as
// launch_x_fwd_list serves it: the list's tiles, or the own launch's grid
int PK_SUFFIX(x_fwd_list_blocks)(const XFwdArgs &a)
{
    int nt = 0, gx = 0;
    size_t b = 0;
    const bool ok = a.residual == 1 ? xr_list_class(a, nt, gx, b) : xf_list_class(a, nt, gx, b);
    return ok ? gx : PK_SUFFIX(x_fwd_grid)(a);
}

}  // namespace pk
