// api.cpp -- C ABI of the FFT-based Poisson solver (declared in
// include/poisson.h): descriptor validation, plan construction (FP64
// twiddle and eigenvalue tables, workspace), the pass sequence of FluTAS
// Section 3.3.1 (forward x, forward y, z solve, backward y, backward x), the
// FP32 + FP64-residual iterative refinement loop, and batched solves in which
// problems of one shape share every launch.
#include "../../include/poisson.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

using namespace pk;

namespace {

// device scalars per problem: [0] mean of f from the zero-wavenumber column,
// [1] sum f, [2] sum r^2, [3] sum (f - mean f)^2, [4] sum p
constexpr int NSCAL = 8;

// ---------------------------------------------------------------------------
// host tables
// ---------------------------------------------------------------------------
// (cos, sin) of 2 pi t / n, reduced to the first octant with exact integer
// arithmetic and evaluated in long double, then rounded once to double.
void cis_2pi(long t, long n, double &c, double &s)
{
    t %= n;
    if (t < 0) t += n;
    const long q = (4 * t) / n;    // quadrant
    const long r = 4 * t - q * n;  // angle within the quadrant = (r/n) pi/2
    long double cc, ss;
    const long double halfpi = 1.5707963267948966192313216916397514L;
    if (2 * r <= n) {
        const long double phi = halfpi * (long double)r / (long double)n;
        cc = cosl(phi);
        ss = sinl(phi);
    } else {
        const long double phi = halfpi * (long double)(n - r) / (long double)n;
        cc = sinl(phi);
        ss = cosl(phi);
    }
    const double c0 = (double)cc, s0 = (double)ss;
    switch (q) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
    }
}

// exp(-2 pi i t/n), t in [0, n), interleaved (re, im)
std::vector<double> twiddle_table(int n)
{
    std::vector<double> tw(2 * (size_t)n);
    for (int t = 0; t < n; ++t) {
        double c, s;
        cis_2pi(t, n, c, s);
        tw[2 * t] = c;
        tw[2 * t + 1] = -s;
    }
    return tw;
}

// lam(j) = -(4/h^2) sin^2(pi j / n): eigenvalues of the periodic 3-point
// second difference (modified wavenumbers), j in [0, count)
std::vector<double> eig_table(int n, double h, int count)
{
    std::vector<double> l(count);
    for (int j = 0; j < count; ++j) {
        double c, s;
        cis_2pi(j, 2L * n, c, s);  // sin(2 pi j / (2n)) = sin(pi j/n)
        l[j] = -4.0 / (h * h) * s * s;
    }
    return l;
}

// eigenvalues of the 3-point operator on n cells between two walls:
// Neumann lam(k) = -(4/h^2) sin^2(pi k/(2n)) (cosine modes), Dirichlet
// lam(k) = -(4/h^2) sin^2(pi (k+1)/(2n)) (sine modes), k in [0, n)
std::vector<double> eig_table_walls(int n, double h, int bc)
{
    std::vector<double> l(n);
    for (int k = 0; k < n; ++k) {
        double c, s;
        cis_2pi(bc == POISSON_BC_DIRICHLET ? k + 1 : k, 4L * n, c, s);
        l[k] = -4.0 / (h * h) * s * s;
    }
    return l;
}

// exp(-i pi k/(2n)), k in [0, n): the half-sample shift of the cosine and
// sine expansions
std::vector<double> quarter_table(int n)
{
    std::vector<double> tw(2 * (size_t)n);
    for (int k = 0; k < n; ++k) {
        double c, s;
        cis_2pi(k, 4L * n, c, s);
        tw[2 * k] = c;
        tw[2 * k + 1] = -s;
    }
    return tw;
}

// Rows of the z system of a stretched grid (cells of thickness h[k]), in the
// form of the z solve (rows multiplied by h[k]), 8 doubles per row:
// {a_k, c_k, h_k, D_k, d_k+1/2, sum_{j<k} h_j, 0, 0}: a_k and c_k the
// conductances 1/d of the faces below and above (d the distance of the two
// cell centres; 0 at a wall), D_k = 2/h_k at a Dirichlet wall (the value is
// zero on the face, half a cell away), d_k+1/2 the centre distance above
// (0 on the last row).  16 padding rows {0, 0, 0, 1, 0, sum h, 0, 0} follow
// (the z solve's last chunk runs past nz).
std::vector<double> zrow_table(const std::vector<double> &h, int bc_z)
{
    const int nz = (int)h.size();
    std::vector<double> t(8 * (size_t)(nz + 16), 0.0);
    double pre = 0.0;
    for (int k = 0; k < nz; ++k) {
        double *r = &t[8 * (size_t)k];
        r[0] = k > 0 ? 1.0 / (0.5 * (h[k - 1] + h[k])) : 0.0;
        r[1] = k < nz - 1 ? 1.0 / (0.5 * (h[k] + h[k + 1])) : 0.0;
        r[2] = h[k];
        if (bc_z == POISSON_BC_DIRICHLET) {
            if (k == 0) r[3] += 2.0 / h[0];
            if (k == nz - 1) r[3] += 2.0 / h[nz - 1];
        }
        r[4] = k < nz - 1 ? 0.5 * (h[k] + h[k + 1]) : 0.0;
        r[5] = pre;
        pre += h[k];
    }
    for (int k = nz; k < nz + 16; ++k) {
        t[8 * (size_t)k + 3] = 1.0;
        t[8 * (size_t)k + 5] = pre;
    }
    return t;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    bool owned = true;  // false: a piece of a region the plan does not own
    ~DevBuf()
    {
        if (p && owned) (void)hipFree(p);
    }
};

struct PinnedBuf {
    void *p = nullptr;
    ~PinnedBuf()
    {
        if (p) (void)hipHostFree(p);
    }
};

bool fail_alloc_hook()
{
    const char *e = getenv("POISSON_TEST_FAIL_ALLOC");
    return e && *e && strcmp(e, "0") != 0;
}

int dev_alloc(std::shared_ptr<DevBuf> &out, size_t bytes)
{
    if (fail_alloc_hook()) return POISSON_ERR_OUT_OF_MEMORY;
    auto b = std::make_shared<DevBuf>();
    if (bytes == 0) bytes = 16;
    if (hipMalloc(&b->p, bytes) != hipSuccess) {
        b->p = nullptr;
        (void)hipGetLastError();
        return POISSON_ERR_OUT_OF_MEMORY;
    }
    out = b;
    return POISSON_OK;
}

int pinned_alloc(std::unique_ptr<PinnedBuf> &out, size_t bytes)
{
    if (fail_alloc_hook()) return POISSON_ERR_OUT_OF_MEMORY;
    out.reset(new PinnedBuf());
    if (hipHostMalloc(&out->p, bytes, 0) != hipSuccess) {
        out->p = nullptr;
        (void)hipGetLastError();
        return POISSON_ERR_OUT_OF_MEMORY;
    }
    memset(out->p, 0, bytes);
    return POISSON_OK;
}

int upload(std::shared_ptr<DevBuf> &out, const void *host, size_t bytes)
{
    int rc = dev_alloc(out, bytes);
    if (rc) return rc;
    if (hipMemcpy(out->p, host, bytes, hipMemcpyHostToDevice) != hipSuccess) return POISSON_ERR_HIP;
    return POISSON_OK;
}

// Where a plan's device memory comes from: its own hipMalloc'd buffers, or
// pieces of one caller-provided region (the allocation-free solve), carved in
// order at 256-byte alignment.  In the region mode the tables are not copied
// one by one: their bytes are staged at the same offsets in a host image of
// the region, which the caller copies to the device in one transfer.
struct Alloc {
    char *base = nullptr;          // null: hipMalloc every buffer
    size_t cap = 0, used = 0;
    std::vector<char> *image = nullptr;  // host image of [base, base + used) for tables

    int get(std::shared_ptr<DevBuf> &out, size_t bytes)
    {
        if (!base) return dev_alloc(out, bytes);
        const size_t off = (used + 255) & ~(size_t)255;
        if (bytes == 0) bytes = 16;
        if (off > cap || bytes > cap - off) return POISSON_ERR_OUT_OF_MEMORY;
        auto b = std::make_shared<DevBuf>();
        b->p = base + off;
        b->owned = false;
        used = off + bytes;
        out = b;
        return POISSON_OK;
    }
    int put(std::shared_ptr<DevBuf> &out, const void *host, size_t bytes)
    {
        if (!base) return upload(out, host, bytes);
        const int rc = get(out, bytes);
        if (rc) return rc;
        const size_t off = (size_t)((char *)out->p - base);
        if (image->size() < off + bytes) image->resize(off + bytes, 0);
        memcpy(image->data() + off, host, bytes);
        return POISSON_OK;
    }
};

int upload_complex(Alloc &A, std::shared_ptr<DevBuf> out[2], const std::vector<double> &tw,
                   bool need32, bool need64)
{
    int rc;
    if (need64 && (rc = A.put(out[0], tw.data(), tw.size() * sizeof(double)))) return rc;
    if (need32) {
        std::vector<float> f(tw.size());
        for (size_t i = 0; i < tw.size(); ++i) f[i] = (float)tw[i];  // one rounding
        if ((rc = A.put(out[1], f.data(), f.size() * sizeof(float)))) return rc;
    }
    return POISSON_OK;
}

// ---------------------------------------------------------------------------
// launch variants (autotuned per shape)
// ---------------------------------------------------------------------------
// zv: tile of the wall-bounded z solve (launch_z_walls), yv: tile / radix
// order of the y passes (YCfg), rev: reversed block order of the passes that
// read what the previous pass just wrote (block_order).
struct Tune {
    int zv = 0, yv = 0, rev = 1;
    int kr = 8;          // z-planes per workgroup of the residual pass with transform
    int krc = 8;         // the same for the residual check (negative: exact depth)
    bool tuned = false;  // chosen by timing (else the defaults below)
};

// Defaults from measurements on MI355X (512x512x256 and 1024x1024x512):
// wide z tiles for FP64 up to 256 planes, narrow beyond; the reverse for FP32.
// POISSON_ZWALLS_VARIANT / POISSON_Y_VARIANT / POISSON_BLOCK_ORDER=forward
// force a choice (measurements).
Tune heuristic_tune(const poisson_desc_t &d)
{
    Tune t;
    const bool f64 = d.precision == POISSON_FP64;
    t.zv = f64 ? (d.nz <= 256 ? 2 : 0) : (d.nz <= 256 ? 0 : 2);
    t.yv = 0;
    t.rev = 1;
    return t;
}

void apply_env_overrides(Tune &t)
{
    if (const char *e = getenv("POISSON_ZWALLS_VARIANT")) t.zv = atoi(e) & 3;
    if (const char *e = getenv("POISSON_Y_VARIANT")) t.yv = atoi(e) & 3;
    if (const char *e = getenv("POISSON_BLOCK_ORDER")) t.rev = strcmp(e, "forward") == 0 ? 0 : 1;
    // plane-range depths of the residual passes: 4, 8 or 16 (halved for
    // small grids), other positive values exact
    auto depth = [](const char *e, int &kr) {
        const int k = atoi(e);
        if (k == 4 || k == 8 || k == 16) kr = k;
        else if (k > 0 && k <= 4096) kr = -k;
    };
    if (const char *e = getenv("POISSON_MARCH_PLANES")) depth(e, t.kr);
    if (const char *e = getenv("POISSON_CHECK_PLANES")) depth(e, t.krc);
}

// process-wide cache of tuned variants: key "precision nx ny nz bc device"
std::mutex tune_mu;
std::map<std::string, Tune> tune_cache;
bool tune_file_loaded = false;

// stretched: the group's z cells are not uniform (the plan keeps them apart
// from the descriptor)
std::string tune_key(const poisson_desc_t &d, bool stretched)
{
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    char buf[160];
    // stretched z grids run other z-solve kernels: their own entries
    snprintf(buf, sizeof buf, "%s %d %d %d %d%d%d%s %s",
             d.precision == POISSON_FP64 ? "f64" : "f32", d.nx, d.ny, d.nz, d.bc_x, d.bc_y,
             d.bc_z, stretched ? "s" : "", arch.c_str());
    for (char *c = buf; *c; ++c)
        if (*c == ':') *c = '_';
    return buf;
}

// optional persistence: POISSON_TUNE_CACHE names a text file of lines
// "<key> : zv yv rev kr krc"
void load_tune_file()
{
    if (tune_file_loaded) return;
    tune_file_loaded = true;
    const char *path = getenv("POISSON_TUNE_CACHE");
    if (!path) return;
    FILE *fp = fopen(path, "r");
    if (!fp) return;
    char line[256];
    while (fgets(line, sizeof line, fp)) {
        char *colon = strchr(line, ':');
        if (!colon) continue;
        *colon = 0;
        std::string key(line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        Tune t;
        const int got = sscanf(colon + 1, "%d %d %d %d %d", &t.zv, &t.yv, &t.rev, &t.kr, &t.krc);
        if (got >= 3) {
            t.zv &= 3;
            t.yv &= 3;
            t.rev = t.rev ? 1 : 0;
            auto ok = [](int k) { return k == 4 || k == 8 || k == 16 || (k < 0 && k >= -4096); };
            if (got < 4 || !ok(t.kr)) t.kr = 8;
            if (got < 5 || !ok(t.krc)) t.krc = t.kr;
            t.tuned = true;
            tune_cache[key] = t;
        }
    }
    fclose(fp);
}

void save_tune_file()
{
    const char *path = getenv("POISSON_TUNE_CACHE");
    if (!path) return;
    FILE *fp = fopen(path, "w");
    if (!fp) return;
    for (auto &kv : tune_cache)
        fprintf(fp, "%s : %d %d %d %d %d\n", kv.first.c_str(), kv.second.zv, kv.second.yv,
                kv.second.rev, kv.second.kr, kv.second.krc);
    fclose(fp);
}

Tune initial_tune(const poisson_desc_t &d, bool stretched)
{
    Tune t = heuristic_tune(d);
    {
        std::lock_guard<std::mutex> lk(tune_mu);
        load_tune_file();
        auto it = tune_cache.find(tune_key(d, stretched));
        if (it != tune_cache.end()) t = it->second;
    }
    apply_env_overrides(t);
    return t;
}

// ---------------------------------------------------------------------------
// plan structures
// ---------------------------------------------------------------------------
struct Tables {
    std::shared_ptr<DevBuf> twx[2], twy[2], twz[2];  // [0] FP64, [1] FP32 complex tables
    std::shared_ptr<DevBuf> twy4[2];                 // walls along y: exp(-i pi k/(2 ny))
    std::shared_ptr<DevBuf> twx4[2];                 // walls along x: exp(-i pi k/(2 nx))
    std::shared_ptr<DevBuf> lamx, lamy, lamz;
    std::shared_ptr<DevBuf> zrow;  // stretched z: the rows of the z system
    std::shared_ptr<DevBuf> hz;    // stretched z: thickness of each plane
    std::shared_ptr<DevBuf> zc;    // stretched z: residual coefficients of each plane
};

// problems with identical descriptors: one set of tables, one launch per pass
struct Group {
    poisson_desc_t d;      // dz_cells is cleared: the thicknesses live in hz
    std::vector<double> hz;  // stretched z: the cell thicknesses (empty: uniform)
    double hsum = 0.0;
    double mean_div = 0.0;   // sums of f and p over this give the (volume-weighted) means
    int M = 0;
    long long N = 0;
    Tables tab;
    std::vector<int> members;          // problem indices in the plan
    std::shared_ptr<DevBuf> S32;       // FP32 spectra, one per member
    std::shared_ptr<DevBuf> P32;       // refinement: FP32 first iterates, one per member
    std::shared_ptr<DevBuf> partials;  // per-workgroup partial sums, part_stride per member
    int npart = 0;                     // workgroups of the forward x pass (upper bound)
    int part_stride = 0;               // doubles of partials per member
    Tune tune;                         // launch variants of this shape (autotuned)
    int host_off = 0;                  // offset of this group's staging entries
};

struct Timed {
    std::string name;
    double bytes;
    hipEvent_t e0, e1;
};

struct PassStat {
    int launches = 0;
    double total_ms = 0.0;
    double bytes = 0.0;
};

// One pass of one shape group, recorded instead of launched (work-list
// schedule): the launches of every group at the same position of their
// sequences are issued together, one work-list launch per pass kind.
enum RecKind { RK_XF, RK_XR, RK_XI, RK_Y, RK_Z, RK_RC, RK_SUM };
struct Rec {
    int kind = RK_XF;
    std::string name;
    double bytes = 0.0;
    XFwdArgs xf{};
    XInvArgs xi{};
    YArgs y{};
    ZArgs z{};
    SumSeg sum{};
};

}  // namespace

struct poisson_plan_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int precision = 0;
    double rtol = 1e-10;
    int max_refine = 8;
    bool batched = false;
    int count = 0;
    std::vector<Group> groups;
    std::vector<std::pair<int, int>> where;  // problem -> (group, member slot)
    std::shared_ptr<DevBuf> scalars;         // NSCAL FP64 scalars per problem
    std::unique_ptr<PinnedBuf> host_scalars;
    void *hs = nullptr;                      // host copy of scalars + control records
    std::unique_ptr<PinnedBuf> host_ptrs;    // ProbPtrs staging for batched launches
    hipEvent_t ptrs_done = nullptr;          // last staging upload has been consumed
    hipStream_t ls = nullptr;                // stream the passes of the current solve use
    // device-side refinement loop (poisson_plan_set_graph): 0 host-driven loop,
    // 1 captured graphs, 2 the same launch sequence issued eagerly
    int graph_mode = 0;
    int *ctrl = nullptr;                     // NCTRL ints per problem (after the scalars)
    int *host_ctrl = nullptr;                // host copy (after the host scalars)
    std::shared_ptr<DevBuf> dptrs;           // ProbPtrs of every problem, by group
    std::vector<ProbPtrs> dptrs_copy;        // what dptrs holds (device-side loop)
    bool dptrs_valid = false;
    hipStream_t gstream = nullptr;           // plan-owned stream of the device loop
    // stream the device loop issues to: the caller's stream (eager launches
    // and graph launches), gstream while a graph is being captured
    hipStream_t ms = nullptr;
    std::vector<hipStream_t> side;           // one more stream per further group
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    hipGraph_t graph[2] = {nullptr, nullptr};  // [0] solve + loop segments, [1] segments
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    // projection step in progress (poisson_project): the first pass takes
    // f = alpha D(u, v, w) instead of reading a right-hand side
    struct Proj {
        const double *u = nullptr, *v = nullptr, *w = nullptr;
        double alpha = 1.0;
        double *f_out = nullptr;  // where the pass stores f (FP32 + refinement)
    } proj;
    bool projecting = false;
    std::shared_ptr<DevBuf> fdiv;  // FP64 f of projections under FP32 + refinement
    // work-list schedule of a batched plan: every pass serves all shape
    // groups in one launch (0: one launch per group, on forked streams)
    bool list_mode = false;
    // the schedule of each refinement-loop driver (host loop; device-side
    // loops), chosen by the autotuner when it runs, and whether an
    // environment setting forces one
    bool list_host = false, list_device = false, sched_forced = false;
    std::vector<Rec> *rec = nullptr;  // non-null: passes are recorded here
    bool timing = false;
    std::vector<Timed> pending;
    std::vector<hipEvent_t> event_pool;
    std::map<std::string, PassStat> stats;

    ~poisson_plan_s()
    {
        for (auto &t : pending) {
            event_pool.push_back(t.e0);
            event_pool.push_back(t.e1);
        }
        for (auto e : event_pool) (void)hipEventDestroy(e);
        if (ptrs_done) (void)hipEventDestroy(ptrs_done);
        drop_graphs();
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        for (auto e : ev_join) (void)hipEventDestroy(e);
        for (auto st : side) (void)hipStreamDestroy(st);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
    void drop_graphs()
    {
        for (int i = 0; i < 2; ++i) {
            if (gexec[i]) (void)hipGraphExecDestroy(gexec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            gexec[i] = nullptr;
            graph[i] = nullptr;
        }
    }
};

namespace {

int validate(const poisson_desc_t *d)
{
    if (!d) return POISSON_ERR_INVALID_ARG;
    if (d->nx < 2 || d->ny < 1 || d->nz < 1) return POISSON_ERR_INVALID_ARG;
    if (!(std::isfinite(d->dx) && d->dx > 0) || !(std::isfinite(d->dy) && d->dy > 0) ||
        !(std::isfinite(d->dz) && d->dz > 0))
        return POISSON_ERR_INVALID_ARG;
    auto known = [](int bc) { return bc >= POISSON_BC_PERIODIC && bc <= POISSON_BC_DIRICHLET; };
    if (!known(d->bc_x) || !known(d->bc_y) || !known(d->bc_z)) return POISSON_ERR_INVALID_ARG;
    if (d->precision < POISSON_FP64 || d->precision > POISSON_FP32) return POISSON_ERR_INVALID_ARG;
    if (d->precision == POISSON_FP32_REFINE) {
        if (!(std::isfinite(d->rtol) && d->rtol > 0)) return POISSON_ERR_INVALID_ARG;
        if (d->max_refine < 1 || d->max_refine > 1000) return POISSON_ERR_INVALID_ARG;
    }
    if (d->nx % 2) return POISSON_ERR_UNSUPPORTED;
    if (d->nx / 2 > 1024 || !fft_length_supported(d->nx / 2)) return POISSON_ERR_UNSUPPORTED;
    if (!fft_length_supported(d->ny)) return POISSON_ERR_UNSUPPORTED;
    if (d->bc_z == POISSON_BC_PERIODIC) {
        if (!fft_length_supported(d->nz)) return POISSON_ERR_UNSUPPORTED;
    } else if (d->nz > 4096) {
        return POISSON_ERR_UNSUPPORTED;
    }
    const long long n = (long long)d->nx * d->ny * d->nz;
    if (n > (1LL << 31)) return POISSON_ERR_UNSUPPORTED;
    if (d->dz_cells) {
        // stretched z: walls in z only, positive finite thicknesses
        if (d->bc_z == POISSON_BC_PERIODIC) return POISSON_ERR_UNSUPPORTED;
        for (int k = 0; k < d->nz; ++k)
            if (!(std::isfinite(d->dz_cells[k]) && d->dz_cells[k] > 0))
                return POISSON_ERR_INVALID_ARG;
    }
    return POISSON_OK;
}

int internal_prec(int precision) { return precision == POISSON_FP64 ? P_F64 : P_F32; }

// bytes of the per-problem state: NSCAL doubles, then NCTRL ints, per problem
size_t state_bytes(int count) { return (NSCAL * sizeof(double) + NCTRL * sizeof(int)) * count; }

// per-workgroup partial-sum records (4 doubles each) a problem needs: the
// largest grid of the passes that write them
int partial_slots(const poisson_desc_t &d)
{
    int n = x_fwd_blocks(internal_prec(d.precision), d.nx, d.ny, d.nz, 0, 0);
    if (d.precision != POISSON_FP64) {
        // residual and divergence passes (plane march): the most workgroups
        // any plane-range depth gives
        const int r = x_fwd_blocks(P_F32, d.nx, d.ny, d.nz, 1, 1);
        n = n > r ? n : r;
    }
    if (d.precision == POISSON_FP32_REFINE) {
        const int c = residual_check_blocks(d.nx, d.ny, d.nz, 1);
        n = n > c ? n : c;
    }
    return n;
}

size_t workspace_bytes(const poisson_desc_t *d)
{
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    size_t b = 0;
    if (d->precision != POISSON_FP64) b += n * 4;  // FP32 half spectrum: N/2 complex floats
    if (d->precision == POISSON_FP32_REFINE) b += n * 4;  // FP32 first iterate
    b += (size_t)partial_slots(*d) * 4 * sizeof(double);
    return b;
}

// a zero-value wall on some axis: the operator has no null space, so no
// mean is removed from f or p
bool regular(const poisson_desc_t &d)
{
    return d.bc_x == POISSON_BC_DIRICHLET || d.bc_y == POISSON_BC_DIRICHLET ||
           d.bc_z == POISSON_BC_DIRICHLET;
}

bool same_problem(const poisson_desc_t &a, const poisson_desc_t &b)
{
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.dx == b.dx && a.dy == b.dy &&
           a.dz == b.dz && a.bc_x == b.bc_x && a.bc_y == b.bc_y && a.bc_z == b.bc_z;
}

// Tables of the group in A (copied now, or staged in A's host image), then
// the field-sized buffers
int build_group(Group &g, Alloc &A)
{
    const poisson_desc_t &d = g.d;
    g.M = d.nx / 2;
    g.N = (long long)d.nx * d.ny * d.nz;
    const bool f32 = d.precision != POISSON_FP64, f64 = !f32;
    int rc;
    Tables &t = g.tab;
    if ((rc = upload_complex(A, t.twx, twiddle_table(d.nx), f32, f64))) return rc;
    if ((rc = upload_complex(A, t.twy, twiddle_table(d.ny), f32, f64))) return rc;
    if (d.bc_z == POISSON_BC_PERIODIC &&
        (rc = upload_complex(A, t.twz, twiddle_table(d.nz), f32, f64)))
        return rc;
    // walls along x: nx cosine / sine modes; periodic: M + 1 wavenumbers
    auto lx = d.bc_x == POISSON_BC_PERIODIC ? eig_table(d.nx, d.dx, g.M + 1)
                                            : eig_table_walls(d.nx, d.dx, d.bc_x);
    if (d.bc_x != POISSON_BC_PERIODIC &&
        (rc = upload_complex(A, t.twx4, quarter_table(d.nx), f32, f64)))
        return rc;
    auto ly = d.bc_y == POISSON_BC_PERIODIC ? eig_table(d.ny, d.dy, d.ny)
                                            : eig_table_walls(d.ny, d.dy, d.bc_y);
    if (d.bc_y != POISSON_BC_PERIODIC &&
        (rc = upload_complex(A, t.twy4, quarter_table(d.ny), f32, f64)))
        return rc;
    auto lz = eig_table(d.nz, d.dz, d.nz);
    g.mean_div = (double)g.N;
    if (!g.hz.empty()) {
        auto zt = zrow_table(g.hz, d.bc_z);
        g.hsum = zt[8 * g.hz.size() + 5];
        g.mean_div = (double)d.nx * d.ny * g.hsum;
        if ((rc = A.put(t.zrow, zt.data(), zt.size() * 8))) return rc;
        if ((rc = A.put(t.hz, g.hz.data(), g.hz.size() * 8))) return rc;
        // residual: (a_k, c_k) / h_k per plane, 1/h_k^2 at a Dirichlet wall
        // (the march's ghost plane is the negated wall plane), 0 at a
        // Neumann wall (the ghost plane mirrors it)
        std::vector<double> zc(2 * g.hz.size());
        for (size_t k = 0; k < g.hz.size(); ++k) {
            const double *r = &zt[8 * k];
            const double hk = g.hz[k];
            const bool wall_lo = k == 0, wall_hi = k + 1 == g.hz.size();
            const bool dir = d.bc_z == POISSON_BC_DIRICHLET;
            zc[2 * k] = wall_lo ? (dir ? 1.0 / (hk * hk) : 0.0) : r[0] / hk;
            zc[2 * k + 1] = wall_hi ? (dir ? 1.0 / (hk * hk) : 0.0) : r[1] / hk;
        }
        if ((rc = A.put(t.zc, zc.data(), zc.size() * 8))) return rc;
    }
    if ((rc = A.put(t.lamx, lx.data(), lx.size() * 8))) return rc;
    if ((rc = A.put(t.lamy, ly.data(), ly.size() * 8))) return rc;
    if ((rc = A.put(t.lamz, lz.data(), lz.size() * 8))) return rc;
    const size_t n = g.members.size();
    g.npart = x_fwd_blocks(internal_prec(d.precision), d.nx, d.ny, d.nz, 0, 0);
    g.part_stride = partial_slots(d) * 4;
    if ((rc = A.get(g.partials, (size_t)g.part_stride * sizeof(double) * n))) return rc;
    if (f32 && (rc = A.get(g.S32, (size_t)g.N * 4 * n))) return rc;
    // the first iterate of the refinement is an FP32 field: kept exactly in
    // 4 B/point, it is written and read back at half the bytes
    const bool refine = d.precision == POISSON_FP32_REFINE;
    if (refine && (rc = A.get(g.P32, (size_t)g.N * 4 * n))) return rc;
    g.tune = initial_tune(g.d, !g.hz.empty());
    return POISSON_OK;
}

// ---------------------------------------------------------------------------
// launch bookkeeping (optional per-pass hipEvent timing)
// ---------------------------------------------------------------------------
// a failed HIP call is reported on stderr with the pass it belongs to
int hip_fail(const char *what, int e)
{
    fprintf(stderr, "libpoisson: %s failed: %s (%d)\n", what,
            e > 0 ? hipGetErrorString((hipError_t)e) : "no kernel for this size", e);
    return POISSON_ERR_HIP;
}

template <class F>
int timed(poisson_plan p, const char *name, double bytes, F &&launch)
{
    if (!p->timing) {
        int e = launch();
        return e ? hip_fail(name, e) : POISSON_OK;
    }
    Timed t{name, bytes, nullptr, nullptr};
    for (hipEvent_t *ev : {&t.e0, &t.e1}) {
        if (!p->event_pool.empty()) {
            *ev = p->event_pool.back();
            p->event_pool.pop_back();
        } else if (hipEventCreate(ev) != hipSuccess) {
            return POISSON_ERR_HIP;
        }
    }
    (void)hipEventRecord(t.e0, p->ls);
    int e = launch();
    (void)hipEventRecord(t.e1, p->ls);
    p->pending.push_back(t);
    return e ? hip_fail(name, e) : POISSON_OK;
}

void collect_timing(poisson_plan p)
{
    if (p->pending.empty()) return;
    (void)hipEventSynchronize(p->pending.back().e1);
    for (auto &t : p->pending) {
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, t.e0, t.e1);
        auto &st = p->stats[t.name];
        st.launches += 1;
        st.total_ms += ms;
        st.bytes = t.bytes;
        p->event_pool.push_back(t.e0);
        p->event_pool.push_back(t.e1);
    }
    p->pending.clear();
}

const char *tag(int prec) { return prec == P_F32 ? "f32" : "f64"; }


// ---------------------------------------------------------------------------
// one pass over a set of problems of one group
// ---------------------------------------------------------------------------
// `dev` null: a single problem with the pointers in `one`; otherwise `n`
// problems whose ProbPtrs are in device memory at `dev`.
struct LSet {
    poisson_plan p;
    Group *g;
    int prec;
    const ProbPtrs *dev;
    int n;
    ProbPtrs one;
    int gate = 0;      // control slot gating the passes (device-side loop)
    int sum_mode = 0;  // control step taken by the sum of the forward x pass
    // refinement: the first solve writes its iterate to the FP32 copy
    // (use32); while the current iterate is that copy (cur32) the residual
    // pass reads it and the next accumulating pass reads it and writes p
    bool use32 = false;
    bool cur32 = false;
};

// problems that share the plane-range choice of the residual passes: the
// whole group in a batched launch, whichever of them a launch still serves;
// in the work-list schedule every problem of the plan (one launch serves
// them all)
int kr_group(const LSet &L)
{
    if (!L.dev) return 1;
    return L.p->list_mode ? L.p->count : (int)L.g->members.size();
}

int pass_x_fwd(LSet &L, bool residual, bool want_partials, bool sum = true)
{
    Group &g = *L.g;
    const double sb = L.prec == P_F32 ? 4.0 : 8.0;
    XFwdArgs a{};
    a.batch = L.dev;
    a.nbatch = L.n;
    a.f = L.one.f;
    a.p = L.one.p;
    a.S = L.one.S;
    a.tw = g.tab.twx[L.prec == P_F32 ? 1 : 0]->p;
    a.partials = want_partials ? (L.dev ? (double *)g.partials->p : L.one.partials) : nullptr;
    a.nx = g.d.nx;
    a.ny = g.d.ny;
    a.nz = g.d.nz;
    a.bc_z = g.d.bc_z;
    a.bc_y = g.d.bc_y;
    a.bc_x = g.d.bc_x;
    a.tw4x = g.d.bc_x != POISSON_BC_PERIODIC ? g.tab.twx4[L.prec == P_F32 ? 1 : 0]->p : nullptr;
    a.ax = 1.0 / (g.d.dx * g.d.dx);
    a.ay = 1.0 / (g.d.dy * g.d.dy);
    a.az = 1.0 / (g.d.dz * g.d.dz);
    a.sum_f = L.one.scal ? L.one.scal + 1 : nullptr;
    a.inv_n = 1.0 / g.mean_div;
    a.hz = g.tab.hz ? (const double *)g.tab.hz->p : nullptr;
    a.zc = g.tab.zc ? (const double *)g.tab.zc->p : nullptr;
    a.residual = residual ? 1 : 0;
    a.gate = L.gate;
    a.kr_max = g.tune.kr;
    a.kr_nb = kr_group(L);
    a.regular = regular(g.d) ? 1 : 0;
    a.p_in32 = residual && L.cur32 ? 1 : 0;
    a.p32 = L.one.p32;
    char name[40];
    snprintf(name, sizeof name, residual ? "x_r2c_residual_%s" : "x_r2c_%s", tag(L.prec));
    double bytes = (double)g.N * ((residual ? (a.p_in32 ? 12.0 : 16.0) : 8.0) + sb) * L.n;
    const bool div = !residual && L.p->projecting;
    if (div) {
        // projection: f = alpha D(u, v, w) evaluated on the fly (one problem)
        const auto &pj = L.p->proj;
        a.residual = 2;
        a.u = pj.u;
        a.v = pj.v;
        a.w = pj.w;
        a.cx = pj.alpha / g.d.dx;
        a.cy = pj.alpha / g.d.dy;
        a.cz = pj.alpha / g.d.dz;
        a.f_out = pj.f_out;
        snprintf(name, sizeof name, "x_r2c_divergence_%s", tag(L.prec));
        bytes = (double)g.N * (24.0 + sb + (pj.f_out ? 8.0 : 0.0)) * L.n;
    }
    int np = 0;
    int rc;
    if (L.p->rec) {
        Rec r;
        r.kind = residual ? RK_XR : RK_XF;
        r.name = name;
        r.bytes = bytes;
        r.xf = a;
        L.p->rec->push_back(r);
        np = x_fwd_list_blocks(L.prec, a);
        rc = np < 0 ? hip_fail(name, -1) : POISSON_OK;
    } else {
        rc = timed(L.p, name, bytes, [&] { return launch_x_fwd(L.prec, a, &np, L.p->ls); });
    }
    if (rc || !want_partials || !sum) return rc;
    // three sums per workgroup: plain input -> (sum f, 0, 0) into scal[1..3];
    // residual -> (sum r^2, sum fbar^2, sum p) into scal[2..4]
    const int off = residual ? 2 : 1;
    if (L.p->rec) {
        Rec r;
        r.kind = RK_SUM;
        r.name = "sum_partials";
        r.bytes = (double)np * 32.0 * L.n;
        r.sum = SumSeg{L.dev, L.n, np, 0, off, 0, L.sum_mode};
        L.p->rec->push_back(r);
        return POISSON_OK;
    }
    return timed(L.p, "sum_partials", (double)np * 32.0 * L.n, [&] {
        return launch_sum_partials(L.one.partials, np, L.one.scal ? L.one.scal + off : nullptr,
                                   L.dev, L.n, off, L.p->ls, 0, L.sum_mode, L.p->rtol,
                                   L.p->max_refine);
    });
}

// residual and its norms without the transform (a convergence check that
// does not write the spectrum): sums into scal[2..4] like the residual x pass
int pass_residual_check(LSet &L, bool sum = true)
{
    Group &g = *L.g;
    // a check follows a correction, which left the iterate in p; the loops
    // never ask for a check of the first iterate
    if (L.cur32) {
        fprintf(stderr, "libpoisson: residual check requested for the FP32 first iterate\n");
        return POISSON_ERR_HIP;
    }
    XFwdArgs a{};
    a.batch = L.dev;
    a.nbatch = L.n;
    a.f = L.one.f;
    a.p = L.one.p;
    a.partials = L.one.partials;
    a.nx = g.d.nx;
    a.ny = g.d.ny;
    a.nz = g.d.nz;
    a.bc_z = g.d.bc_z;
    a.bc_y = g.d.bc_y;
    a.bc_x = g.d.bc_x;
    a.ax = 1.0 / (g.d.dx * g.d.dx);
    a.ay = 1.0 / (g.d.dy * g.d.dy);
    a.az = 1.0 / (g.d.dz * g.d.dz);
    a.sum_f = L.one.scal ? L.one.scal + 1 : nullptr;
    a.inv_n = 1.0 / g.mean_div;
    a.hz = g.tab.hz ? (const double *)g.tab.hz->p : nullptr;
    a.zc = g.tab.zc ? (const double *)g.tab.zc->p : nullptr;
    a.residual = 1;
    a.gate = L.gate;
    a.kr_max = g.tune.krc;
    a.kr_nb = kr_group(L);
    a.regular = regular(g.d) ? 1 : 0;
    int nc = 0;
    int rc;
    if (L.p->rec) {
        Rec r;
        r.kind = RK_RC;
        r.name = "residual_check_f64";
        r.bytes = (double)g.N * 16.0 * L.n;
        r.xf = a;
        L.p->rec->push_back(r);
        nc = residual_check_blocks(a.nx, a.ny, a.nz, a.kr_max, a.kr_nb);
        rc = POISSON_OK;
    } else {
        rc = timed(L.p, "residual_check_f64", (double)g.N * 16.0 * L.n,
                   [&] { return launch_residual_check(a, &nc, L.p->ls); });
    }
    if (rc || !sum) return rc;
    if (L.p->rec) {
        Rec r;
        r.kind = RK_SUM;
        r.name = "sum_partials";
        r.bytes = (double)nc * 32.0 * L.n;
        r.sum = SumSeg{L.dev, L.n, nc, 0, 2, 0, 0};
        L.p->rec->push_back(r);
        return POISSON_OK;
    }
    return timed(L.p, "sum_partials", (double)nc * 32.0 * L.n, [&] {
        return launch_sum_partials(L.one.partials, nc, L.one.scal ? L.one.scal + 2 : nullptr,
                                   L.dev, L.n, 2, L.p->ls);
    });
}

int pass_y(LSet &L, bool inverse)
{
    Group &g = *L.g;
    // a length-1 transform is the identity (recorded all the same, so that
    // every group's sequence has the same passes; the list launcher skips it)
    if (g.d.ny == 1 && !L.p->rec) return POISSON_OK;
    // the forward y pass follows the x pass, which wrote the planes in order
    const int pi = L.prec == P_F32 ? 1 : 0;
    const bool wall = g.d.bc_y != POISSON_BC_PERIODIC;
    YArgs a{L.dev, L.n, L.one.S, g.tab.twy[pi]->p, g.M, g.d.ny, g.d.nz,
            inverse ? 1 : 0, (!inverse && g.tune.rev) ? 1 : 0, L.gate, g.tune.yv,
            g.d.bc_y, wall ? g.tab.twy4[pi]->p : nullptr};
    char name[40];
    snprintf(name, sizeof name, inverse ? "y_inv_%s" : "y_fwd_%s", tag(L.prec));
    const double bytes = (double)g.N * 2.0 * (L.prec == P_F32 ? 4.0 : 8.0) * L.n;
    if (L.p->rec) {
        Rec r;
        r.kind = RK_Y;
        r.name = name;
        r.bytes = g.d.ny == 1 ? 0.0 : bytes;
        r.y = a;
        L.p->rec->push_back(r);
        return POISSON_OK;
    }
    return timed(L.p, name, bytes, [&] { return launch_y(L.prec, a, L.p->ls); });
}

int pass_z(LSet &L)
{
    Group &g = *L.g;
    ZArgs a{};
    a.batch = L.dev;
    a.nbatch = L.n;
    a.S = L.one.S;
    a.tw = g.d.bc_z == POISSON_BC_PERIODIC ? g.tab.twz[L.prec == P_F32 ? 1 : 0]->p : nullptr;
    a.lamx = (const double *)g.tab.lamx->p;
    a.lamy = (const double *)g.tab.lamy->p;
    a.lamz = (const double *)g.tab.lamz->p;
    // non-null requests the mean; batched launches redirect it per problem
    a.zero_mean_out = L.dev ? (double *)g.partials->p : L.one.scal;
    a.M = g.M;
    a.ny = g.d.ny;
    a.nz = g.d.nz;
    a.nx = g.d.nx;
    a.dz2 = g.d.dz * g.d.dz;
    a.inv_nxny = 1.0 / ((double)g.d.nx * g.d.ny);
    a.inv_ntot = 1.0 / (double)g.N;
    a.variant = g.tune.zv;
    a.gate = L.gate;
    a.dirichlet_z = g.d.bc_z == POISSON_BC_DIRICHLET ? 1 : 0;
    a.regular = regular(g.d) ? 1 : 0;
    a.ywall = g.d.bc_y != POISSON_BC_PERIODIC ? 1 : 0;
    a.xwall = g.d.bc_x != POISSON_BC_PERIODIC ? 1 : 0;
    a.periodic_z = g.d.bc_z == POISSON_BC_PERIODIC ? 1 : 0;
    a.zrow = g.tab.zrow ? (const double *)g.tab.zrow->p : nullptr;
    a.hsum = g.hsum;
    const double bytes = (double)g.N * 2.0 * (L.prec == P_F32 ? 4.0 : 8.0) * L.n;
    char name[40];
    if (L.p->rec) {
        Rec r;
        r.kind = RK_Z;
        snprintf(name, sizeof name, "z_%s", tag(L.prec));
        r.name = name;
        r.bytes = bytes;
        r.z = a;
        L.p->rec->push_back(r);
        return POISSON_OK;
    }
    if (g.d.bc_z != POISSON_BC_PERIODIC) {
        snprintf(name, sizeof name, "z_walls_%s", tag(L.prec));
        return timed(L.p, name, bytes, [&] { return launch_z_walls(L.prec, a, L.p->ls); });
    }
    snprintf(name, sizeof name, "z_periodic_%s", tag(L.prec));
    return timed(L.p, name, bytes, [&] { return launch_z_periodic(L.prec, a, L.p->ls); });
}

int pass_x_inv(LSet &L, bool accumulate)
{
    Group &g = *L.g;
    // the inverse x pass follows the inverse y pass, which wrote the planes in order
    XInvArgs a{L.dev, L.n, L.one.S, L.one.p, g.tab.twx[L.prec == P_F32 ? 1 : 0]->p, g.d.nx,
               g.d.ny, g.d.nz, accumulate ? 1 : 0, g.tune.rev, nullptr,
               1.0 / g.mean_div, L.gate, regular(g.d) ? 1 : 0, g.d.bc_x,
               g.d.bc_x != POISSON_BC_PERIODIC ? g.tab.twx4[L.prec == P_F32 ? 1 : 0]->p
                                               : nullptr,
               0, L.one.p32};
    // the plain pass of the first solve writes the FP32 copy; the first
    // accumulating pass reads it
    const bool in32 = accumulate ? L.cur32 : L.use32;
    a.p_in32 = in32 ? 1 : 0;
    // the mean of p from the residual pass (batched launches redirect it)
    if (accumulate) a.sum_p = L.dev ? (const double *)g.partials->p : L.one.scal + 4;
    char name[40];
    snprintf(name, sizeof name, accumulate ? "x_c2r_accumulate_%s" : "x_c2r_%s", tag(L.prec));
    const double sb = L.prec == P_F32 ? 4.0 : 8.0;
    const double pin = in32 ? 4.0 : 8.0;  // bytes of the iterate read or written in FP32 / FP64
    const double bytes = (double)g.N * (sb + (accumulate ? pin + 8.0 : pin)) * L.n;
    int rc = POISSON_OK;
    if (L.p->rec) {
        Rec r;
        r.kind = RK_XI;
        r.name = name;
        r.bytes = bytes;
        r.xi = a;
        L.p->rec->push_back(r);
    } else {
        rc = timed(L.p, name, bytes, [&] { return launch_x_inv(L.prec, a, L.p->ls); });
    }
    if (!rc) L.cur32 = accumulate ? false : in32;
    return rc;
}

// transform of the right-hand side (or residual), z solve, inverse transform
int solve_passes(LSet &L, bool accumulate_into_p, bool want_partials)
{
    int rc;
    if ((rc = pass_x_fwd(L, false, want_partials))) return rc;
    if ((rc = pass_y(L, false))) return rc;
    if ((rc = pass_z(L))) return rc;
    if ((rc = pass_y(L, true))) return rc;
    return pass_x_inv(L, accumulate_into_p);
}

int correction_passes(LSet &L)
{
    int rc;
    if ((rc = pass_y(L, false))) return rc;
    if ((rc = pass_z(L))) return rc;
    if ((rc = pass_y(L, true))) return rc;
    return pass_x_inv(L, true);
}

// Issue the recorded passes of several groups: position by position (every
// group records the same sequence of pass kinds, or at one position one of
// two kinds), one work-list launch per pass kind present at a position.
int issue_recs(poisson_plan p, std::vector<std::vector<Rec>> &per)
{
    size_t len = 0;
    for (auto &v : per) len = std::max(len, v.size());
    const int prec = internal_prec(p->precision);
    for (size_t i = 0; i < len; ++i) {
        for (int kind = RK_XF; kind <= RK_SUM; ++kind) {
            std::vector<const Rec *> rs;
            for (auto &v : per)
                if (i < v.size() && v[i].kind == kind) rs.push_back(&v[i]);
            if (rs.empty()) continue;
            double bytes = 0.0;
            for (auto *r : rs) bytes += r->bytes;
            const int n = (int)rs.size();
            const char *name = rs[0]->name.c_str();
            int rc = POISSON_OK;
            switch (kind) {
            case RK_XF:
            case RK_XR: {
                std::vector<XFwdArgs> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->xf;
                rc = timed(p, name, bytes,
                           [&] { return launch_x_fwd_list(prec, a.data(), n, p->ls); });
                break;
            }
            case RK_XI: {
                std::vector<XInvArgs> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->xi;
                rc = timed(p, name, bytes,
                           [&] { return launch_x_inv_list(prec, a.data(), n, p->ls); });
                break;
            }
            case RK_Y: {
                std::vector<YArgs> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->y;
                rc = timed(p, name, bytes, [&] { return launch_y_list(prec, a.data(), n, p->ls); });
                break;
            }
            case RK_Z: {
                std::vector<ZArgs> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->z;
                rc = timed(p, name, bytes, [&] { return launch_z_list(prec, a.data(), n, p->ls); });
                break;
            }
            case RK_RC: {
                std::vector<XFwdArgs> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->xf;
                rc = timed(p, name, bytes,
                           [&] { return launch_residual_check_list(a.data(), n, p->ls); });
                break;
            }
            default: {
                std::vector<SumSeg> a(n);
                for (int k = 0; k < n; ++k) a[k] = rs[k]->sum;
                rc = timed(p, name, bytes, [&] {
                    return launch_sum_partials_list(a.data(), n, p->rtol, p->max_refine, p->ls);
                });
                break;
            }
            }
            if (rc) return rc;
        }
    }
    return POISSON_OK;
}

// Run f (the passes of one group) for the listed groups: launched group by
// group, or, in the work-list schedule, recorded for every group and then
// issued together.
template <class F>
int over_groups(poisson_plan p, std::vector<LSet> &sets, const std::vector<size_t> &which, F &&f)
{
    if (!p->list_mode) {
        for (size_t gi : which) {
            const int rc = f(sets[gi]);
            if (rc) return rc;
        }
        return POISSON_OK;
    }
    // the groups of the largest problems first: their blocks are dispatched
    // first and the small problems' blocks fill the end of each launch
    std::vector<size_t> order(which);
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t a, size_t b) { return sets[a].g->N > sets[b].g->N; });
    std::vector<std::vector<Rec>> per(order.size());
    int rc = POISSON_OK;
    for (size_t k = 0; k < order.size() && !rc; ++k) {
        p->rec = &per[k];
        rc = f(sets[order[k]]);
    }
    p->rec = nullptr;
    return rc ? rc : issue_recs(p, per);
}

int read_scalars(poisson_plan p, int count)
{
    hipError_t e = hipMemcpyAsync(p->hs, p->scalars->p, NSCAL * sizeof(double) * count,
                                  hipMemcpyDeviceToHost, p->ls);
    if (e != hipSuccess) return hip_fail("scalar read-back", (int)e);
    e = hipStreamSynchronize(p->ls);
    if (e != hipSuccess) return hip_fail("stream synchronize", (int)e);
    return POISSON_OK;
}

// [a, a + na) and [b, b + nb) (doubles) share a byte
bool overlaps(const double *a, long long na, const double *b, long long nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + (uintptr_t)(nb * 8) && y < x + (uintptr_t)(na * 8);
}

// pointers of problem i (member slot `slot` of group g)
ProbPtrs problem_ptrs(poisson_plan p, const Group &g, int slot, const double *rhs, double *sol)
{
    const int i = g.members[slot];
    ProbPtrs q;
    q.f = rhs;
    q.p = sol;
    q.S = p->precision == POISSON_FP64
              ? (void *)sol
              : (void *)((char *)g.S32->p + (size_t)g.N * 4 * slot);
    q.partials = (double *)g.partials->p + (size_t)g.part_stride * slot;
    q.scal = (double *)p->scalars->p + NSCAL * i;
    q.ctrl = p->ctrl + NCTRL * i;
    q.p32 = g.P32 ? (float *)((char *)g.P32->p + (size_t)g.N * 4 * slot) : nullptr;
    return q;
}

enum { RUNNING = 1, DONE = 0 };

// Solve every problem of the plan.  Single-problem plans launch with direct
// pointers; batched plans upload one ProbPtrs array per group and launch
// each pass once per group.  FP32 + refinement synchronises once per
// iteration for the whole plan.
int solve_all(poisson_plan p, const double *const *rhs, double *const *sol, poisson_stats_t *st)
{
    p->list_mode = p->list_host;
    const int prec = internal_prec(p->precision);
    const int count = p->count;
    std::vector<LSet> sets(p->groups.size());
    std::vector<std::vector<int>> active(p->groups.size());
    ProbPtrs *staging = p->batched ? (ProbPtrs *)p->host_ptrs->p : nullptr;
    p->ls = p->stream;

    // (re)write the device pointer arrays for the listed member slots
    auto stage = [&](int gi) -> int {
        Group &g = p->groups[gi];
        LSet &L = sets[gi];
        L.n = (int)active[gi].size();
        if (!p->batched) {
            L.dev = nullptr;
            L.one = problem_ptrs(p, g, 0, rhs[0], sol[0]);
            return POISSON_OK;
        }
        ProbPtrs *h = staging + g.host_off;
        for (int k = 0; k < L.n; ++k) {
            const int slot = active[gi][k];
            const int i = g.members[slot];
            h[k] = problem_ptrs(p, g, slot, rhs[i], sol[i]);
        }
        L.dev = (const ProbPtrs *)p->dptrs->p + g.host_off;
        L.one = ProbPtrs{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        p->dptrs_valid = false;
        if (L.n == 0) return POISSON_OK;
        hipError_t e = hipMemcpyAsync((ProbPtrs *)p->dptrs->p + g.host_off, h,
                                      sizeof(ProbPtrs) * L.n, hipMemcpyHostToDevice, p->ls);
        return e == hipSuccess ? POISSON_OK : hip_fail("pointer upload", (int)e);
    };

    if (p->batched && p->ptrs_done) {
        // the staging area may still feed the previous call's copies
        if (hipEventSynchronize(p->ptrs_done) != hipSuccess) return POISSON_ERR_HIP;
    }
    int rc = POISSON_OK;
    for (size_t gi = 0; gi < p->groups.size() && !rc; ++gi) {
        sets[gi] = LSet{p, &p->groups[gi], prec, nullptr, 0, {}};
        sets[gi].use32 = p->groups[gi].P32 != nullptr;
        active[gi].resize(p->groups[gi].members.size());
        for (size_t k = 0; k < active[gi].size(); ++k) active[gi][k] = (int)k;
        rc = stage((int)gi);
    }

    std::vector<poisson_stats_t> out(count, poisson_stats_t{0, -1.0, 0.0, POISSON_OK});
    const bool refine = p->precision == POISSON_FP32_REFINE;
    const bool want_partials = prec == P_F32;  // FP64 mean comes from the z pass
    std::vector<size_t> all(p->groups.size());
    for (size_t gi = 0; gi < all.size(); ++gi) all[gi] = gi;
    if (!rc)
        rc = over_groups(p, sets, all,
                         [&](LSet &L) { return solve_passes(L, false, want_partials); });

    if (!rc && refine) {
        std::vector<double> rho_prev(count, -1.0), rho_first(count, -1.0);
        std::vector<int> corrections(count, 0), state(count, RUNNING);
        std::vector<char> checked(p->groups.size(), 0);
        double *hs = (double *)p->hs;
        for (int it = 0; !rc; ++it) {
            // Residual of every running problem.  Each correction multiplies
            // the residual by about the relative accuracy of the FP32 solve,
            // i.e. by the first residual rho_first; when rho_prev * rho_first
            // is two decades below rtol for every running problem of a group,
            // its residual is only checked (no transform, no spectrum write).
            // If the check fails, the full residual pass follows.
            std::vector<size_t> running;
            for (size_t gi = 0; gi < p->groups.size(); ++gi) {
                checked[gi] = 0;
                if (!sets[gi].n) continue;
                bool predict = true;
                for (int slot : active[gi]) {
                    const int i = p->groups[gi].members[slot];
                    predict = predict && rho_first[i] > 0 && rho_prev[i] > 0 &&
                              rho_prev[i] * rho_first[i] * 100.0 <= p->rtol;
                }
                checked[gi] = predict;
                running.push_back(gi);
            }
            rc = over_groups(p, sets, running, [&](LSet &L) {
                const size_t gi = (size_t)(L.g - p->groups.data());
                return checked[gi] ? pass_residual_check(L) : pass_x_fwd(L, true, true);
            });
            if (rc || (rc = read_scalars(p, count))) break;
            std::vector<size_t> fix;
            bool any = false;
            for (size_t gi = 0; gi < p->groups.size(); ++gi) {
                std::vector<int> next;
                for (int slot : active[gi]) {
                    const int i = p->groups[gi].members[slot];
                    const double *s = hs + NSCAL * i;
                    const double rho = s[3] > 0 ? std::sqrt(s[2] / s[3]) : std::sqrt(s[2]);
                    out[i].rel_residual = rho;
                    out[i].rhs_mean = regular(p->groups[gi].d) ? 0.0 : s[1] / p->groups[gi].mean_div;
                    out[i].iterations = corrections[i];
                    int status = -1;
                    if (!std::isfinite(rho))
                        status = POISSON_ERR_NONFINITE;
                    else if (rho <= p->rtol)
                        status = POISSON_OK;
                    else if (corrections[i] >= p->max_refine ||
                             (rho_prev[i] >= 0 && rho > 0.5 * rho_prev[i]))
                        status = POISSON_ERR_NOT_CONVERGED;
                    if (rho_first[i] < 0) rho_first[i] = rho;
                    if (status != -1) {
                        out[i].status = status;
                        state[i] = DONE;
                        // stopped before any correction: the solution is the
                        // first iterate, still in its FP32 copy
                        if (sets[gi].cur32 && !rc) {
                            const ProbPtrs q =
                                problem_ptrs(p, p->groups[gi], slot, rhs[i], sol[i]);
                            const int e = launch_widen(q.p32, sol[i],
                                                       (size_t)p->groups[gi].N, p->ls);
                            if (e) rc = hip_fail("first iterate widening", e);
                        }
                    } else {
                        rho_prev[i] = rho;
                        corrections[i] += 1;
                        next.push_back(slot);
                    }
                }
                if (next.size() != active[gi].size()) {
                    active[gi] = next;
                    if ((rc = stage((int)gi))) break;
                }
                // a check-only pass wrote no spectrum: transform the residual
                // of the problems that go on
                if (checked[gi] && !next.empty()) fix.push_back(gi);
                any = any || !next.empty();
            }
            if (!rc && !fix.empty())
                rc = over_groups(p, sets, fix, [&](LSet &L) { return pass_x_fwd(L, true, true); });
            if (rc || !any) break;
            std::vector<size_t> go;
            for (size_t gi = 0; gi < p->groups.size(); ++gi)
                if (sets[gi].n) go.push_back(gi);
            rc = over_groups(p, sets, go, [&](LSet &L) { return correction_passes(L); });
        }
    } else if (!rc && st) {
        rc = read_scalars(p, count);
        const double *hs = (const double *)p->hs;
        for (auto &g : p->groups)
            for (int i : g.members)
                out[i].rhs_mean =
                    regular(g.d) ? 0.0
                                 : (prec == P_F64 ? hs[NSCAL * i] : hs[NSCAL * i + 1] / g.mean_div);
    }
    if (p->batched && p->ptrs_done) (void)hipEventRecord(p->ptrs_done, p->ls);

    int first = rc;
    for (int i = 0; i < count; ++i) {
        if (rc) out[i].status = rc;
        if (!first && out[i].status) first = out[i].status;
        if (st) st[i] = out[i];
    }
    return first;
}

// ---------------------------------------------------------------------------
// device-side refinement loop (poisson_plan_set_graph)
// ---------------------------------------------------------------------------
// Loop segments per graph: one correction (when the control kernel says so)
// followed by the residual evaluation that decides on the next.  A problem
// that needs more corrections gets further launches of the segment-only
// graph.
constexpr int GRAPH_SEGMENTS = 2;
// segments after the head: a problem that converges after one correction
// (the usual case) ends the first round with no gated-off launch but the
// unused kind of residual pass
constexpr int HEAD_SEGMENTS = 1;

// full residual pass [C_FULL] | residual check [C_CHECK, optional]
// | sums + control decision [C_EVAL]
int enqueue_residual_decision(poisson_plan p, LSet &L, bool with_check)
{
    Group &g = *L.g;
    int rc;
    L.gate = C_FULL;
    if ((rc = pass_x_fwd(L, true, true, false))) return rc;
    if (with_check) {
        L.gate = C_CHECK;
        if ((rc = pass_residual_check(L, false))) return rc;
    }
    // partial records of whichever residual pass ran for each problem
    const int nr = x_fwd_blocks(P_F32, g.d.nx, g.d.ny, g.d.nz, 1, g.tune.kr, kr_group(L));
    const int nc = residual_check_blocks(g.d.nx, g.d.ny, g.d.nz, g.tune.krc, kr_group(L));
    if (p->rec) {
        Rec r;
        r.kind = RK_SUM;
        r.name = "sum_partials";
        r.bytes = (double)(nr > nc ? nr : nc) * 32.0 * L.n;
        r.sum = SumSeg{L.dev, L.n, nr, nc, 2, C_EVAL, 2};
        p->rec->push_back(r);
        L.gate = 0;
        return POISSON_OK;
    }
    rc = timed(p, "sum_partials", (double)(nr > nc ? nr : nc) * 32.0 * L.n, [&] {
        return launch_sum_partials(nullptr, nr, nullptr, L.dev, L.n, 2, p->ls, C_EVAL, 2,
                                   p->rtol, p->max_refine, nc);
    });
    L.gate = 0;
    return rc;
}

// The launch sequence of the device-side loop for one group, on the stream
// p->ls.  head: the first solve, whose sum of f also opens the control
// records, and the first residual (always the full pass); then segments of
//   full residual pass after a failed check [C_FIX]
//   | y, z, y, accumulating x [C_CORRECT]
//   | full residual pass [C_FULL] | residual check [C_CHECK]
//   | sums + control decision [C_EVAL]
// (HEAD_SEGMENTS after the head, GRAPH_SEGMENTS otherwise).  The first
// segment after the head has no fix: the decision before it followed a
// full residual pass.
int enqueue_group_sequence(poisson_plan p, LSet &L, bool head, bool segs = true)
{
    const bool refine = p->precision == POISSON_FP32_REFINE;
    const int prec = internal_prec(p->precision);
    int rc = POISSON_OK;
    if (head) {
        L.gate = 0;
        L.sum_mode = refine ? 1 : 0;
        rc = solve_passes(L, false, prec == P_F32);
        L.sum_mode = 0;
        if (rc) return rc;
    }
    if (!refine || !segs) return POISSON_OK;
    if (head && (rc = enqueue_residual_decision(p, L, false))) return rc;
    const int nseg = head ? HEAD_SEGMENTS : GRAPH_SEGMENTS;
    for (int seg = 0; seg < nseg; ++seg) {
        if (!(head && seg == 0)) {
            L.gate = C_FIX;
            if ((rc = pass_x_fwd(L, true, true, false))) return rc;
        }
        L.gate = C_CORRECT;
        if ((rc = correction_passes(L))) return rc;
        if ((rc = enqueue_residual_decision(p, L, true))) return rc;
    }
    L.gate = 0;
    return POISSON_OK;
}

// All groups, each on a stream of its own forked from the plan's loop
// stream and joined back (in a captured graph: independent branches), so
// that the launches of problems of different shapes overlap.  The host
// issues the groups with the most points first: the longest sequence starts
// while the launches of the others are still being issued.
int enqueue_device_sequence(poisson_plan p, std::vector<LSet> &sets, bool head,
                            bool segs = true)
{
    const size_t ng = sets.size();
    int rc = POISSON_OK;
    if (p->list_mode) {
        // work-list schedule: every group's sequence recorded, then issued
        // on the loop stream, one launch per pass for all groups
        p->ls = p->ms;
        std::vector<size_t> all(ng);
        for (size_t gi = 0; gi < ng; ++gi) all[gi] = gi;
        return over_groups(p, sets, all,
                           [&](LSet &L) { return enqueue_group_sequence(p, L, head, segs); });
    }
    std::vector<size_t> order(ng);
    for (size_t gi = 0; gi < ng; ++gi) order[gi] = gi;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const Group &ga = *sets[a].g, &gb = *sets[b].g;
        return (double)ga.N * ga.members.size() > (double)gb.N * gb.members.size();
    });
    if (ng > 1 && hipEventRecord(p->ev_fork, p->ms) != hipSuccess)
        return hip_fail("stream fork", (int)hipGetLastError());
    for (size_t oi = 0; oi < ng && !rc; ++oi) {
        const size_t gi = order[oi];
        p->ls = gi == 0 ? p->ms : p->side[gi - 1];
        if (gi > 0 && hipStreamWaitEvent(p->ls, p->ev_fork, 0) != hipSuccess) {
            rc = hip_fail("stream fork", (int)hipGetLastError());
            break;
        }
        rc = enqueue_group_sequence(p, sets[gi], head, segs);
        if (gi > 0 && hipEventRecord(p->ev_join[gi - 1], p->ls) != hipSuccess && !rc)
            rc = hip_fail("stream join", (int)hipGetLastError());
    }
    p->ls = p->ms;
    for (size_t gi = 1; gi < ng; ++gi)
        if (hipStreamWaitEvent(p->ms, p->ev_join[gi - 1], 0) != hipSuccess && !rc)
            rc = hip_fail("stream join", (int)hipGetLastError());
    return rc;
}

int ensure_device_loop_objects(poisson_plan p)
{
    if (p->gstream) return POISSON_OK;
    // streams of default priority (non-blocking: ordered by events only)
    if (hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) != hipSuccess) {
        p->gstream = nullptr;
        return POISSON_ERR_HIP;
    }
    auto ev = [](hipEvent_t *e) {
        return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    };
    if (!ev(&p->ev_fork)) return POISSON_ERR_HIP;
    for (size_t gi = 1; gi < p->groups.size(); ++gi) {
        hipStream_t st = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return POISSON_ERR_HIP;
        p->side.push_back(st);
        if (!ev(&e)) return POISSON_ERR_HIP;
        p->ev_join.push_back(e);
    }
    return POISSON_OK;
}

// capture the sequence into graph k (0: head + segments, 1: segments)
int build_graph(poisson_plan p, std::vector<LSet> &sets, int k)
{
    hipError_t e = hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail("graph capture", (int)e);
    hipStream_t ms = p->ms;
    p->ms = p->gstream;
    const int rc = enqueue_device_sequence(p, sets, k == 0);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->gstream, &g);
    p->ms = ms;
    if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return rc ? rc : hip_fail("graph capture", (int)e);
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail("graph instantiate", (int)e);
    }
    p->graph[k] = g;
    p->gexec[k] = x;
    return POISSON_OK;
}

// Solve with the device-side loop on the caller's stream: per round one
// graph launch (or the same launches issued eagerly) and one read-back of
// the scalars and control records.
int solve_device(poisson_plan p, const double *const *rhs, double *const *sol,
                 poisson_stats_t *st)
{
    if (p->list_mode != p->list_device) p->drop_graphs();  // captured with the other schedule
    p->list_mode = p->list_device;
    int rc = ensure_device_loop_objects(p);
    if (rc) return rc;
    const int prec = internal_prec(p->precision);
    const bool refine = p->precision == POISSON_FP32_REFINE;
    const bool capture = p->graph_mode == 1 && !p->timing;
    const int count = p->count;
    // launches (eager ones and graph launches) go straight to the caller's
    // stream: ordering a stream of the plan's own after it with an event
    // pair left the GPU idle for 60-85 us between solves on MI355X; graphs
    // are captured on the plan's stream (the caller's may not be capturable)
    p->ms = p->stream;
    p->ls = p->ms;
    if (p->ptrs_done && hipEventSynchronize(p->ptrs_done) != hipSuccess) return POISSON_ERR_HIP;

    // pointers of every problem, uploaded in one copy when they changed
    std::vector<LSet> sets(p->groups.size());
    ProbPtrs *staging = (ProbPtrs *)p->host_ptrs->p;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        Group &g = p->groups[gi];
        const int n = (int)g.members.size();
        for (int k = 0; k < n; ++k) {
            const int i = g.members[k];
            staging[g.host_off + k] = problem_ptrs(p, g, k, rhs[i], sol[i]);
        }
        sets[gi] = LSet{p, &g, prec, (const ProbPtrs *)p->dptrs->p + g.host_off, n, {}};
        // the projection under capture issues its first solve eagerly and
        // continues with the segment-only graph, which reads the iterate in p
        sets[gi].use32 = g.P32 != nullptr && !(capture && p->projecting);
    }
    if (!p->dptrs_valid ||
        memcmp(p->dptrs_copy.data(), staging, sizeof(ProbPtrs) * count) != 0) {
        if (hipMemcpyAsync(p->dptrs->p, staging, sizeof(ProbPtrs) * count, hipMemcpyHostToDevice,
                           p->ms) != hipSuccess)
            return hip_fail("pointer upload", (int)hipGetLastError());
        memcpy(p->dptrs_copy.data(), staging, sizeof(ProbPtrs) * count);
        p->dptrs_valid = true;
    }
    const double *hs = (const double *)p->hs;
    const int *hc = p->host_ctrl;
    const int max_rounds = p->max_refine / GRAPH_SEGMENTS + 2;
    for (int round = 0; !rc; ++round) {
        int k = round == 0 ? 0 : 1;
        bool issued = false;
        if (capture && round == 0 && p->projecting) {
            // the first pass of a projection takes the call's velocity
            // pointers: the solve is issued eagerly, the loop segments come
            // from the segment graph
            if ((rc = enqueue_device_sequence(p, sets, true, false))) break;
            issued = !refine;
            k = 1;
        }
        if (issued) {
        } else if (capture) {
            if (!p->gexec[k] && (rc = build_graph(p, sets, k))) break;
            const hipError_t e = hipGraphLaunch(p->gexec[k], p->ms);
            if (e != hipSuccess) {
                rc = hip_fail("graph launch", (int)e);
                break;
            }
        } else if ((rc = enqueue_device_sequence(p, sets, round == 0))) {
            break;
        }
        if (!refine && !st) break;
        // scalars and control records are one allocation: one read-back
        if (hipMemcpyAsync(p->hs, p->scalars->p, state_bytes(count),
                           hipMemcpyDeviceToHost, p->ms) != hipSuccess ||
            hipStreamSynchronize(p->ms) != hipSuccess) {
            rc = hip_fail("scalar read-back", (int)hipGetLastError());
            break;
        }
        if (!refine) break;
        bool running = false;
        for (int i = 0; i < count; ++i) running = running || hc[NCTRL * i + C_STATE] != 0;
        if (!running || round + 1 >= max_rounds) break;
    }
    if (p->ptrs_done) (void)hipEventRecord(p->ptrs_done, p->ms);

    int first = rc;
    for (auto &g : p->groups) {
        for (int i : g.members) {
            poisson_stats_t o{0, -1.0, 0.0, POISSON_OK};
            if (!rc && (refine || st)) {
                const double *sc = hs + NSCAL * i;
                const int *c = hc + NCTRL * i;
                o.rhs_mean = regular(g.d) ? 0.0 : (prec == P_F64 ? sc[0] : sc[1] / g.mean_div);
                if (refine) {
                    o.rel_residual = sc[5];
                    o.iterations = c[C_CORR];
                    o.status = c[C_STATE] ? POISSON_ERR_NOT_CONVERGED : c[C_STATUS];
                }
            }
            if (rc) o.status = rc;
            if (!first && o.status) first = o.status;
            if (st) st[i] = o;
        }
    }
    return first;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
// Times the launch variants of one shape group on scratch fields of that
// shape (one problem, zero data: the passes are bandwidth-bound and take no
// data-dependent paths) and keeps the fastest, one knob after the other: the
// z-solve tile, the y tile and radix order, the block order.  Each candidate
// is scored on the whole pass sequence (one warm-up, then the mean of three).
int autotune_group(poisson_plan p, Group &g)
{
    const int prec = internal_prec(p->precision);
    std::shared_ptr<DevBuf> f, sol, scal;
    int rc;
    if ((rc = dev_alloc(f, (size_t)g.N * 8)) || (rc = dev_alloc(sol, (size_t)g.N * 8)) ||
        (rc = dev_alloc(scal, NSCAL * 8)))
        return rc;
    if (hipMemsetAsync(f->p, 0, (size_t)g.N * 8, p->stream) != hipSuccess ||
        hipMemsetAsync(sol->p, 0, (size_t)g.N * 8, p->stream) != hipSuccess ||
        hipMemsetAsync(scal->p, 0, NSCAL * 8, p->stream) != hipSuccess ||
        (g.S32 && hipMemsetAsync(g.S32->p, 0, (size_t)g.N * 4, p->stream) != hipSuccess))
        return hip_fail("autotune scratch", (int)hipGetLastError());
    void *S = prec == P_F64 ? sol->p : g.S32->p;
    ProbPtrs one{(const double *)f->p, (double *)sol->p, S, (double *)g.partials->p,
                 (double *)scal->p, nullptr};
    LSet L{p, &g, prec, nullptr, 1, one};
    p->ls = p->stream;
    const bool timing = p->timing;
    p->timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        p->timing = timing;
        return POISSON_ERR_HIP;
    }
    auto measure = [&](auto &&fn) -> double {
        if (fn()) return -1.0;
        (void)hipEventRecord(e0, p->stream);
        for (int i = 0; i < 3; ++i)
            if (fn()) return -1.0;
        (void)hipEventRecord(e1, p->stream);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 3.0;
    };
    auto pick = [&](int &knob, int n, auto &&fn) {
        int best = knob;
        double bt = 1e300;
        for (int v = 0; v < n; ++v) {
            knob = v;
            const double t = measure(fn);
            if (t >= 0.0 && t < bt) {
                bt = t;
                best = v;
            }
        }
        knob = best;
    };
    // every candidate is scored on the whole pass sequence: how fast a pass
    // runs depends on how much of its input the previous pass left in the
    // last-level cache
    auto whole = [&] { return solve_passes(L, false, false); };
    if (g.d.bc_z != POISSON_BC_PERIODIC) pick(g.tune.zv, 4, whole);
    if (g.d.ny >= 64) pick(g.tune.yv, g.d.bc_y == POISSON_BC_PERIODIC ? 4 : 2, whole);
    pick(g.tune.rev, 2, whole);
    if (p->precision == POISSON_FP32_REFINE) {
        // plane-range depths of the residual pass with transform and of the
        // residual check, each scored on its own pass: 4, 8 or 16 planes
        // (halved for small grids), and the exact depths whose workgroups
        // fill the device's resident slots in one or two whole rounds (a
        // last partial round leaves most of the device idle: 1024 workgroups
        // of 16 planes on 768 slots at 512x512x256 ran 6 % slower than 1536
        // of 22)
        // The candidates are timed on one problem of the group's shape, so
        // the exact depths are offered to single-problem groups only (for a
        // batched group they would be sized for one problem and run with all
        // of them)
        const bool single = g.members.size() <= 1;
        auto candidates = [&](int njb, int slots, int *c) {
            int n = 0;
            for (int k : {4, 8, 16}) c[n++] = k;
            for (int rounds = 1; single && rounds <= 2 && slots > 0 && njb > 0; ++rounds) {
                const long want = (long)slots * rounds / (long)njb;
                if (want < 1) continue;
                const int kr = (int)((g.d.nz + want - 1) / want);
                bool dup = false;
                for (int i = 0; i < n; ++i) dup = dup || c[i] == -kr;
                if (!dup) c[n++] = -kr;
            }
            return n;
        };
        int cr[5], cc[5];
        const int xw = g.d.bc_x != POISSON_BC_PERIODIC ? 1 : 0;
        const int nr = candidates(x_fwd_blocks(P_F32, g.d.nx, g.d.ny, g.d.nz, 1, -g.d.nz, 1),
                                  x_res_slots(g.d.nx, xw, L.cur32 ? 1 : 0), cr);
        const int nc = candidates(residual_check_blocks(g.d.nx, g.d.ny, g.d.nz, -g.d.nz, 1),
                                  residual_check_slots(g.d.nx), cc);
        int idx = 1;
        pick(idx, nr, [&] {
            g.tune.kr = cr[idx];
            return pass_x_fwd(L, true, true);
        });
        g.tune.kr = cr[idx];
        idx = 1;
        pick(idx, nc, [&] {
            g.tune.krc = cc[idx];
            return pass_residual_check(L);
        });
        g.tune.krc = cc[idx];
    }
    g.tune.tuned = true;
    (void)hipStreamSynchronize(p->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->timing = timing;
    return POISSON_OK;
}

// Schedule of a batch of several shapes (work list or per-group launches),
// per loop driver: each candidate times the whole batched solve on zero
// scratch fields (first solve, residual and the control decision), one
// warm-up and then the mean of three.
int autotune_schedule(poisson_plan p)
{
    if (!p->batched || p->groups.size() < 2 || p->sched_forced) return POISSON_OK;
    size_t total = 0;
    for (auto &g : p->groups) total += (size_t)g.N * g.members.size();
    std::shared_ptr<DevBuf> fbuf, sbuf;
    int rc;
    if ((rc = dev_alloc(fbuf, total * 8)) || (rc = dev_alloc(sbuf, total * 8))) return rc;
    if ((rc = launch_zero(fbuf->p, total * 8, p->stream)))
        return hip_fail("autotune scratch", rc);
    std::vector<const double *> rhs(p->count);
    std::vector<double *> sol(p->count);
    size_t off = 0;
    for (auto &g : p->groups)
        for (int i : g.members) {
            rhs[i] = (const double *)fbuf->p + off;
            sol[i] = (double *)sbuf->p + off;
            off += (size_t)g.N;
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return POISSON_ERR_HIP;
    const int mode0 = p->graph_mode;
    const bool timing = p->timing;
    p->timing = false;
    auto run = [&](int mode) {
        p->graph_mode = mode;
        return mode ? solve_device(p, rhs.data(), sol.data(), nullptr)
                    : solve_all(p, rhs.data(), sol.data(), nullptr);
    };
    auto measure = [&](int mode) -> double {
        if (run(mode) < 0) return -1.0;
        (void)hipStreamSynchronize(p->stream);
        (void)hipEventRecord(e0, p->stream);
        for (int i = 0; i < 3; ++i)
            if (run(mode) < 0) return -1.0;
        (void)hipEventRecord(e1, p->stream);
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms / 3.0;
    };
    for (int mode : {0, 2}) {
        bool &knob = mode ? p->list_device : p->list_host;
        knob = false;
        const double tg = measure(mode);
        knob = true;
        const double tl = measure(mode);
        knob = !(tg >= 0.0 && (tl < 0.0 || tg < tl));
    }
    p->graph_mode = mode0;
    p->timing = timing;
    p->drop_graphs();
    (void)hipStreamSynchronize(p->stream);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return POISSON_OK;
}

int autotune_plan(poisson_plan p, int flags)
{
    int rc = POISSON_OK;
    for (auto &g : p->groups) {
        const std::string key = tune_key(g.d, !g.hz.empty());
        bool cached = false;
        if (!(flags & POISSON_TUNE_FORCE)) {
            std::lock_guard<std::mutex> lk(tune_mu);
            load_tune_file();
            auto it = tune_cache.find(key);
            if (it != tune_cache.end() && it->second.tuned) {
                g.tune = it->second;
                cached = true;
            }
        }
        if (!cached) {
            if ((rc = autotune_group(p, g))) return rc;
            std::lock_guard<std::mutex> lk(tune_mu);
            tune_cache[key] = g.tune;
            save_tune_file();
        }
        apply_env_overrides(g.tune);
    }
    p->drop_graphs();  // launch shapes may have changed
    return autotune_schedule(p);
}

int create_plan(const poisson_desc_t *descs, int count, void *stream, bool batched,
                poisson_plan *out)
{
    if (!descs || !out || count < 1) return POISSON_ERR_INVALID_ARG;
    for (int i = 0; i < count; ++i) {
        int rc = validate(&descs[i]);
        if (rc) return rc;
    }
    std::unique_ptr<poisson_plan_s> p(new poisson_plan_s());
    p->stream = (hipStream_t)stream;
    p->precision = descs[0].precision;
    p->rtol = descs[0].rtol;
    p->max_refine = descs[0].max_refine;
    p->batched = batched;
    p->count = count;
    if (hipGetDevice(&p->device) != hipSuccess) return POISSON_ERR_HIP;
    p->where.resize(count);
    for (int i = 0; i < count; ++i) {
        poisson_desc_t d = descs[i];
        d.precision = p->precision;
        d.rtol = p->rtol;
        d.max_refine = p->max_refine;
        std::vector<double> hz;
        if (d.dz_cells) hz.assign(d.dz_cells, d.dz_cells + d.nz);
        d.dz_cells = nullptr;
        int gi = -1;
        for (size_t k = 0; k < p->groups.size(); ++k)
            if (same_problem(p->groups[k].d, d) && p->groups[k].hz == hz) gi = (int)k;
        if (gi < 0) {
            p->groups.emplace_back();
            p->groups.back().d = d;
            p->groups.back().hz = hz;
            gi = (int)p->groups.size() - 1;
        }
        p->where[i] = {gi, (int)p->groups[gi].members.size()};
        p->groups[gi].members.push_back(i);
    }
    int off = 0;
    for (auto &g : p->groups) {
        Alloc A;
        int rc = build_group(g, A);
        if (rc) return rc;
        g.host_off = off;
        off += (int)g.members.size();
    }
    // scalars, then the control records, in one allocation (and one pinned copy)
    int rc = dev_alloc(p->scalars, state_bytes(count));
    if (rc) return rc;
    if (hipMemset(p->scalars->p, 0, state_bytes(count)) != hipSuccess) return POISSON_ERR_HIP;
    if ((rc = pinned_alloc(p->host_scalars, state_bytes(count)))) return rc;
    p->hs = p->host_scalars->p;
    p->ctrl = (int *)((double *)p->scalars->p + NSCAL * count);
    p->host_ctrl = (int *)((double *)p->hs + NSCAL * count);
    // pointer arrays of batched launches and of the device-side loop
    if ((rc = dev_alloc(p->dptrs, sizeof(ProbPtrs) * count))) return rc;
    p->dptrs_copy.resize(count);
    if ((rc = pinned_alloc(p->host_ptrs, sizeof(ProbPtrs) * count))) return rc;
    if (hipEventCreateWithFlags(&p->ptrs_done, hipEventDisableTiming) != hipSuccess)
        return POISSON_ERR_HIP;
    // batches of several shapes: one work-list launch per pass serves them
    // all, unless POISSON_BATCH_SCHEDULE=groups asks for one launch per
    // shape group on forked streams
    const char *sched = getenv("POISSON_BATCH_SCHEDULE");
    p->list_mode = batched && p->groups.size() > 1 && !(sched && strcmp(sched, "groups") == 0);
    p->list_host = p->list_device = p->list_mode;
    p->sched_forced = sched && *sched;
    if (const char *e = getenv("POISSON_AUTOTUNE")) {
        if (*e && strcmp(e, "0") != 0 && (rc = autotune_plan(p.get(), 0))) return rc;
    }
    *out = p.release();
    return POISSON_OK;
}

// Projection step (poisson_project): the first pass evaluates
// f = alpha D(u, v, w) on the fly; L psi = f is solved as by poisson_solve;
// after a successful solve one pass applies u -= beta G psi and p += psi.
int project(poisson_plan p, double *u, double *v, double *w, double *pr, double *psi,
            double alpha, double beta, poisson_stats_t *st)
{
    Group &g = p->groups[0];
    const bool refine = p->precision == POISSON_FP32_REFINE;
    if (refine && !p->fdiv) {
        // the residuals of the refinement need f: stored by the first pass
        const int rc = dev_alloc(p->fdiv, (size_t)g.N * sizeof(double));
        if (rc) return rc;
    }
    p->proj.u = u;
    p->proj.v = v;
    p->proj.w = w;
    p->proj.alpha = alpha;
    p->proj.f_out = refine ? (double *)p->fdiv->p : nullptr;
    p->projecting = true;
    // a direct solve reads no right-hand side after its first pass
    const double *rhs = refine ? (const double *)p->fdiv->p : u;
    int rc = p->graph_mode ? solve_device(p, &rhs, &psi, st) : solve_all(p, &rhs, &psi, st);
    p->projecting = false;
    p->proj = poisson_plan_s::Proj{};
    if (rc) return rc;
    CorrArgs a{psi, u, v, w, pr, g.d.nx, g.d.ny, g.d.nz, g.d.bc_z,
               beta / g.d.dx, beta / g.d.dy, beta / g.d.dz, g.tune.kr > 0 ? g.tune.kr : 0,
               g.d.bc_x != POISSON_BC_PERIODIC ? 1 : 0, g.d.bc_y != POISSON_BC_PERIODIC ? 1 : 0};
    p->ls = p->stream;
    const double bytes = (double)g.N * (pr ? 72.0 : 56.0);
    return timed(p, "correct_f64", bytes, [&] { return launch_correct(a, p->stream); });
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            (void)hipSetDevice(dev);
        } else {
            prev = -1;
        }
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

// ---------------------------------------------------------------------------
// allocation-free solve (poisson_solve_noalloc)
// ---------------------------------------------------------------------------
// Every device buffer of the allocation-free entry point -- twiddle and
// eigenvalue tables, partial-sum records, scalars and control records, the
// FP32 spectrum and the FP32 first iterate -- is a piece of this array.  Each
// GPU the library runs on holds its own copy for the life of the process.
// Host code never passes the array's name to a kernel or a copy: it uses the
// device address hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) char scratch[POISSON_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;

// per device: the scratch array's address and a host-side plan whose buffers
// are pieces of it, kept while calls pass the same descriptor
struct NoAllocDevice {
    std::mutex mu;
    char *base = nullptr;
    std::unique_ptr<poisson_plan_s> plan;
    poisson_desc_t desc{};
    std::vector<char> image;  // host image of the table region
    std::vector<double> host_state;
    std::vector<double> hz;   // cell thicknesses of the cached plan (stretched z)
};
NoAllocDevice noalloc_dev[NOALLOC_MAX_DEVICES];

bool same_desc(const poisson_desc_t &a, const poisson_desc_t &b)
{
    return same_problem(a, b) && a.precision == b.precision && a.rtol == b.rtol &&
           a.max_refine == b.max_refine;
}

// The plan of descriptor d inside the scratch array of device D: tables,
// partial sums, the FP32 fields, then the scalars and control records; the
// tables are copied in one transfer on `stream`, which is then synchronised
// (the host image must outlive the copy).  Fails with TOO_LARGE, before any
// copy, when the pieces do not fit.
int noalloc_build(NoAllocDevice &D, const poisson_desc_t &d, int dev, hipStream_t stream)
{
    D.plan.reset();
    std::unique_ptr<poisson_plan_s> p(new poisson_plan_s());
    p->stream = stream;
    p->device = dev;
    p->precision = d.precision;
    p->rtol = d.rtol;
    p->max_refine = d.max_refine;
    p->batched = false;
    p->count = 1;
    p->where.assign(1, {0, 0});
    p->groups.emplace_back();
    Group &g = p->groups.back();
    g.d = d;
    g.d.dz_cells = nullptr;
    if (d.dz_cells) g.hz.assign(d.dz_cells, d.dz_cells + d.nz);
    g.members.assign(1, 0);
    D.image.clear();
    Alloc A;
    A.base = D.base;
    A.cap = POISSON_NOALLOC_SCRATCH_BYTES;
    A.image = &D.image;
    int rc = build_group(g, A);
    if (!rc) rc = A.get(p->scalars, state_bytes(1));
    if (rc == POISSON_ERR_OUT_OF_MEMORY) {
        fprintf(stderr,
                "libpoisson: poisson_solve_noalloc: %dx%dx%d (%s) needs more than the %zu bytes "
                "of its fixed scratch\n",
                d.nx, d.ny, d.nz,
                d.precision == POISSON_FP64 ? "fp64"
                                            : (d.precision == POISSON_FP32 ? "fp32" : "fp32_refine"),
                (size_t)POISSON_NOALLOC_SCRATCH_BYTES);
        return POISSON_ERR_TOO_LARGE;
    }
    if (rc) return rc;
    if (!D.image.empty()) {
        hipError_t e = hipMemcpyAsync(D.base, D.image.data(), D.image.size(),
                                      hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail("scratch table upload", (int)e);
    }
    D.host_state.assign((state_bytes(1) + sizeof(double) - 1) / sizeof(double), 0.0);
    p->hs = D.host_state.data();
    p->ctrl = (int *)((double *)p->scalars->p + NSCAL);
    p->host_ctrl = (int *)((double *)p->hs + NSCAL);
    D.hz = p->groups[0].hz;
    D.plan = std::move(p);
    D.desc = d;
    D.desc.dz_cells = nullptr;
    return POISSON_OK;
}

int solve_noalloc(const poisson_desc_t *d, void *stream, const double *rhs, double *sol,
                  poisson_stats_t *stats)
{
    if (!d || !rhs || !sol) return POISSON_ERR_INVALID_ARG;
    int rc = validate(d);
    if (rc) return rc;
    const long long n = (long long)d->nx * d->ny * d->nz;
    if (overlaps(rhs, n, sol, n)) return POISSON_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hip_fail("hipGetDevice", (int)hipGetLastError());
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return POISSON_ERR_UNSUPPORTED;
    NoAllocDevice &D = noalloc_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if (!D.base) {
        // once per device, with the device current: the address of this
        // device's copy of the scratch array
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail("scratch symbol address", (int)e);
        D.base = (char *)ptr;
    }
    const hipStream_t s = (hipStream_t)stream;
    bool same = D.plan && same_desc(D.desc, *d) && D.hz.size() == (size_t)(d->dz_cells ? d->nz : 0);
    if (same && d->dz_cells)
        same = std::equal(D.hz.begin(), D.hz.end(), d->dz_cells);
    if (!same) {
        if ((rc = noalloc_build(D, *d, dev, s))) {
            D.plan.reset();
            return rc;
        }
    }
    poisson_plan_s *p = D.plan.get();
    p->stream = s;
    // the array keeps the previous call's contents: clear the scalars and
    // control records (the other pieces are written before they are read)
    const int e = launch_zero(p->scalars->p, state_bytes(1), s);
    if (e) return hip_fail("scratch clear", e);
    return solve_all(p, &rhs, &sol, stats);
}

}  // namespace

extern "C" {

int poisson_desc_init(poisson_desc_t *d)
{
    if (!d) return POISSON_ERR_INVALID_ARG;
    memset(d, 0, sizeof *d);
    d->dx = d->dy = d->dz = 1.0;
    d->bc_x = d->bc_y = d->bc_z = POISSON_BC_PERIODIC;
    d->precision = POISSON_FP64;
    d->rtol = 1e-10;
    d->max_refine = 8;
    return POISSON_OK;
}

int poisson_desc_validate(const poisson_desc_t *d) { return validate(d); }

size_t poisson_workspace_bytes(const poisson_desc_t *d)
{
    if (validate(d) != POISSON_OK) return 0;
    return workspace_bytes(d);
}

int poisson_plan_create(const poisson_desc_t *d, void *stream, poisson_plan *out)
{
    return create_plan(d, 1, stream, false, out);
}

int poisson_batch_plan_create(const poisson_desc_t *descs, int count, void *stream,
                              poisson_plan *out)
{
    return create_plan(descs, count, stream, true, out);
}

int poisson_solve(poisson_plan plan, const double *rhs, double *sol, poisson_stats_t *stats)
{
    if (!plan || !rhs || !sol || plan->batched) return POISSON_ERR_INVALID_ARG;
    const long long n = plan->groups[0].N;
    if (overlaps(rhs, n, sol, n)) return POISSON_ERR_INVALID_ARG;
    DeviceGuard guard(plan->device);
    return plan->graph_mode ? solve_device(plan, &rhs, &sol, stats)
                            : solve_all(plan, &rhs, &sol, stats);
}

int poisson_solve_noalloc(const poisson_desc_t *d, void *stream, const double *rhs, double *sol,
                          poisson_stats_t *stats)
{
    return solve_noalloc(d, stream, rhs, sol, stats);
}

int poisson_batch_solve(poisson_plan plan, const double *const *rhs, double *const *sol,
                        poisson_stats_t *stats)
{
    if (!plan || !rhs || !sol || !plan->batched) return POISSON_ERR_INVALID_ARG;
    // every solution is written while every right-hand side is still read
    // (the refinement's residual passes re-read f): no solution may share a
    // byte with another solution or with any right-hand side
    for (int i = 0; i < plan->count; ++i)
        if (!rhs[i] || !sol[i]) return POISSON_ERR_INVALID_ARG;
    for (int i = 0; i < plan->count; ++i) {
        const long long ni = plan->groups[plan->where[i].first].N;
        for (int j = 0; j < plan->count; ++j) {
            const long long nj = plan->groups[plan->where[j].first].N;
            if (overlaps(sol[i], ni, rhs[j], nj)) return POISSON_ERR_INVALID_ARG;
            if (j < i && overlaps(sol[i], ni, sol[j], nj)) return POISSON_ERR_INVALID_ARG;
        }
    }
    DeviceGuard guard(plan->device);
    return plan->graph_mode ? solve_device(plan, rhs, sol, stats) : solve_all(plan, rhs, sol, stats);
}

int poisson_project(poisson_plan plan, double *u, double *v, double *w, double *p, double *psi,
                    double alpha, double beta, poisson_stats_t *stats)
{
    if (!plan || plan->batched || !u || !v || !w || !psi) return POISSON_ERR_INVALID_ARG;
    if (!std::isfinite(alpha) || !std::isfinite(beta)) return POISSON_ERR_INVALID_ARG;
    // the velocity conventions at the walls are those of the no-slip walls
    // (zero-gradient pressure); zero-value pressure walls are not projected
    const poisson_desc_t &d0 = plan->groups[0].d;
    if (regular(d0) || !plan->groups[0].hz.empty()) return POISSON_ERR_UNSUPPORTED;
    const long long n = plan->groups[0].N;
    const double *arr[5] = {u, v, w, psi, p};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < i; ++j)
            if (arr[i] && arr[j] && overlaps(arr[i], n, arr[j], n)) return POISSON_ERR_INVALID_ARG;
    DeviceGuard guard(plan->device);
    return project(plan, u, v, w, p, psi, alpha, beta, stats);
}

int poisson_plan_autotune(poisson_plan plan, int flags)
{
    if (!plan || (flags & ~POISSON_TUNE_FORCE)) return POISSON_ERR_INVALID_ARG;
    DeviceGuard guard(plan->device);
    (void)hipStreamSynchronize(plan->gstream ? plan->gstream : plan->stream);
    return autotune_plan(plan, flags);
}

int poisson_plan_describe(poisson_plan plan, char *buf, int len)
{
    if (!plan || !buf || len < 1) return POISSON_ERR_INVALID_ARG;
    std::string out;
    char line[256];
    if (plan->batched) {
        snprintf(line, sizeof line,
                 "schedule=%s (host loop: %s, device loops: %s; list = one work-list launch "
                 "per pass for all shapes, groups = one launch per shape group and pass)\n",
                 plan->list_host ? "list" : "groups", plan->list_host ? "list" : "groups",
                 plan->list_device ? "list" : "groups");
        out += line;
    }
    for (size_t gi = 0; gi < plan->groups.size(); ++gi) {
        const Group &g = plan->groups[gi];
        snprintf(line, sizeof line,
                 "group %zu: %dx%dx%d %s %s problems=%zu z_tile=%d y_tile=%d reverse=%d "
                 "march_planes=%d check_planes=%d %s\n",
                 gi,
                 g.d.nx, g.d.ny, g.d.nz,
                 g.d.bc_z == POISSON_BC_NEUMANN
                     ? "walls"
                     : (g.d.bc_z == POISSON_BC_DIRICHLET ? "dirichlet-walls" : "periodic"),
                 plan->precision == POISSON_FP64 ? "fp64"
                                                 : (plan->precision == POISSON_FP32 ? "fp32"
                                                                                     : "fp32_refine"),
                 g.members.size(), g.tune.zv, g.tune.yv, g.tune.rev, std::abs(g.tune.kr),
                 std::abs(g.tune.krc), g.tune.tuned ? "tuned" : "default");
        out += line;
    }
    snprintf(buf, (size_t)len, "%s", out.c_str());
    return (int)out.size() < len ? POISSON_OK : POISSON_ERR_INVALID_ARG;
}

int poisson_plan_set_graph(poisson_plan plan, int mode)
{
    if (!plan || mode < 0 || mode > 2) return POISSON_ERR_INVALID_ARG;
    DeviceGuard guard(plan->device);
    if (mode != plan->graph_mode) {
        // graphs capture the plan's buffers, not the solve's arguments, so they
        // stay valid across solves; a mode change rebuilds them when needed
        (void)hipStreamSynchronize(plan->gstream ? plan->gstream : plan->stream);
        plan->drop_graphs();
    }
    plan->graph_mode = mode;
    return POISSON_OK;
}

int poisson_destroy(poisson_plan plan)
{
    if (!plan) return POISSON_OK;
    (void)hipStreamSynchronize(plan->stream);
    if (plan->gstream) (void)hipStreamSynchronize(plan->gstream);
    delete plan;
    return POISSON_OK;
}

const char *poisson_error_string(int code)
{
    switch (code) {
    case POISSON_OK: return "success";
    case POISSON_ERR_INVALID_ARG: return "invalid argument";
    case POISSON_ERR_UNSUPPORTED: return "unsupported size or boundary combination";
    case POISSON_ERR_OUT_OF_MEMORY: return "device allocation failed";
    case POISSON_ERR_HIP: return "HIP runtime error";
    case POISSON_ERR_NOT_CONVERGED: return "iterative refinement did not converge";
    case POISSON_ERR_NONFINITE: return "non-finite residual";
    case POISSON_ERR_TOO_LARGE: return "problem exceeds the fixed scratch of the allocation-free solve";
    default: return "unknown error code";
    }
}

int poisson_plan_set_timing(poisson_plan plan, int enable)
{
    if (!plan) return POISSON_ERR_INVALID_ARG;
    if (!enable) collect_timing(plan);
    plan->timing = enable != 0;
    return POISSON_OK;
}

int poisson_plan_reset_timing(poisson_plan plan)
{
    if (!plan) return POISSON_ERR_INVALID_ARG;
    collect_timing(plan);
    plan->stats.clear();
    return POISSON_OK;
}

int poisson_plan_get_timing(poisson_plan plan, poisson_pass_stat_t *out, int capacity, int *count)
{
    if (!plan || !count || (capacity > 0 && !out)) return POISSON_ERR_INVALID_ARG;
    collect_timing(plan);
    int i = 0;
    for (auto &kv : plan->stats) {
        if (i < capacity) {
            memset(&out[i], 0, sizeof out[i]);
            snprintf(out[i].name, sizeof out[i].name, "%s", kv.first.c_str());
            out[i].launches = kv.second.launches;
            out[i].total_ms = kv.second.total_ms;
            out[i].bytes_per_launch = kv.second.bytes;
        }
        ++i;
    }
    *count = i;
    return POISSON_OK;
}

}  // extern "C"
