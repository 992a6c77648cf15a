// api.cpp -- C ABI of the FFT-based Poisson solver (declared in
// include/poisson.h): descriptor validation, plan construction (FP64
// twiddle and eigenvalue tables, workspace), the pass sequence of FluTAS
// Section 3.3.1 (forward x, forward y, z solve, backward y, backward x) and
// the FP32 + FP64-residual iterative refinement loop.
#include "../../include/poisson.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"

using namespace pk;

namespace {

// ---------------------------------------------------------------------------
// host tables
// ---------------------------------------------------------------------------
// (cos, sin) of 2 pi t / n, reduced to the first octant with exact integer
// arithmetic and evaluated in long double, then rounded once to double.
void cis_2pi(long t, long n, double &c, double &s)
{
    t %= n;
    if (t < 0) t += n;
    const long q = (4 * t) / n;          // quadrant
    const long r = 4 * t - q * n;        // angle within quadrant = (r/n) pi/2
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
    double c0 = (double)cc, s0 = (double)ss;
    switch (q) {
    case 0: c = c0; s = s0; break;
    case 1: c = -s0; s = c0; break;
    case 2: c = -c0; s = -s0; break;
    default: c = s0; s = -c0; break;
    }
}

// exp(-2 pi i t/n), t in [0, n)
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

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

struct Tables {
    // complex twiddle tables per precision (index 0 = f64, 1 = f32)
    std::shared_ptr<DevBuf> twx[2], twy[2], twz[2];
    std::shared_ptr<DevBuf> lamx, lamy, lamz;
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

struct Sub {
    poisson_desc_t d;
    int M = 0;
    long long N = 0;
    Tables tab;
    std::shared_ptr<DevBuf> S32;  // FP32 spectrum (FP32 modes)
    std::shared_ptr<DevBuf> partials;
    int npart = 0;
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

int upload(std::shared_ptr<DevBuf> &out, const void *host, size_t bytes)
{
    int rc = dev_alloc(out, bytes);
    if (rc) return rc;
    if (hipMemcpy(out->p, host, bytes, hipMemcpyHostToDevice) != hipSuccess) return POISSON_ERR_HIP;
    return POISSON_OK;
}

int upload_complex(std::shared_ptr<DevBuf> out[2], const std::vector<double> &tw, bool need32,
                   bool need64)
{
    int rc;
    if (need64 && (rc = upload(out[0], tw.data(), tw.size() * sizeof(double)))) return rc;
    if (need32) {
        std::vector<float> f(tw.size());
        for (size_t i = 0; i < tw.size(); ++i) f[i] = (float)tw[i];  // one rounding
        if ((rc = upload(out[1], f.data(), f.size() * sizeof(float)))) return rc;
    }
    return POISSON_OK;
}

}  // namespace

struct poisson_plan_s {
    hipStream_t stream = nullptr;
    int device = 0;
    int precision = 0;
    double rtol = 1e-10;
    int max_refine = 8;
    std::vector<Sub> subs;
    std::shared_ptr<DevBuf> scalars;   // device FP64 scalars, 4 per sub
    double *host_scalars = nullptr;    // pinned mirror
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
        if (host_scalars) (void)hipHostFree(host_scalars);
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
    if (d->bc_x != POISSON_BC_PERIODIC || d->bc_y != POISSON_BC_PERIODIC) {
        if ((d->bc_x == POISSON_BC_NEUMANN || d->bc_x == POISSON_BC_PERIODIC) &&
            (d->bc_y == POISSON_BC_NEUMANN || d->bc_y == POISSON_BC_PERIODIC))
            return POISSON_ERR_UNSUPPORTED;
        return POISSON_ERR_INVALID_ARG;
    }
    if (d->bc_z != POISSON_BC_PERIODIC && d->bc_z != POISSON_BC_NEUMANN)
        return POISSON_ERR_INVALID_ARG;
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
    return POISSON_OK;
}

size_t workspace_bytes(const poisson_desc_t *d)
{
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    size_t b = 0;
    if (d->precision != POISSON_FP64) b += n * 4;  // FP32 half spectrum: N/2 complex floats
    const int nb = x_fwd_blocks(d->precision == POISSON_FP64 ? P_F64 : P_F32, d->nx, d->ny, d->nz);
    b += (size_t)(nb > 0 ? nb : 1) * 2 * sizeof(double);
    return b;
}

int build_sub(Sub &s, const poisson_desc_t &d, std::map<std::string, Tables> &cache)
{
    s.d = d;
    s.M = d.nx / 2;
    s.N = (long long)d.nx * d.ny * d.nz;
    const bool f32 = d.precision != POISSON_FP64;
    const bool f64 = d.precision == POISSON_FP64;
    char key[256];
    snprintf(key, sizeof key, "%d %d %d %.17g %.17g %.17g %d %d", d.nx, d.ny, d.nz, d.dx, d.dy,
             d.dz, d.bc_z, d.precision);
    auto it = cache.find(key);
    int rc;
    if (it != cache.end()) {
        s.tab = it->second;
    } else {
        Tables t;
        if ((rc = upload_complex(t.twx, twiddle_table(d.nx), f32, f64))) return rc;
        if ((rc = upload_complex(t.twy, twiddle_table(d.ny), f32, f64))) return rc;
        if (d.bc_z == POISSON_BC_PERIODIC &&
            (rc = upload_complex(t.twz, twiddle_table(d.nz), f32, f64)))
            return rc;
        auto lx = eig_table(d.nx, d.dx, s.M + 1);
        auto ly = eig_table(d.ny, d.dy, d.ny);
        auto lz = eig_table(d.nz, d.dz, d.nz);
        if ((rc = upload(t.lamx, lx.data(), lx.size() * 8))) return rc;
        if ((rc = upload(t.lamy, ly.data(), ly.size() * 8))) return rc;
        if ((rc = upload(t.lamz, lz.data(), lz.size() * 8))) return rc;
        cache[key] = t;
        s.tab = t;
    }
    if (f32 && (rc = dev_alloc(s.S32, (size_t)s.N * 4))) return rc;
    s.npart = x_fwd_blocks(f32 ? P_F32 : P_F64, d.nx, d.ny, d.nz);
    if ((rc = dev_alloc(s.partials, (size_t)s.npart * 2 * sizeof(double)))) return rc;
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
    (void)hipEventRecord(t.e0, p->stream);
    int e = launch();
    (void)hipEventRecord(t.e1, p->stream);
    p->pending.push_back(t);
    return e ? hip_fail(name, e) : POISSON_OK;
}

void collect_timing(poisson_plan p)
{
    if (p->pending.empty()) return;
    (void)hipStreamSynchronize(p->stream);
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
// the pass sequence of one solve
// ---------------------------------------------------------------------------
struct SolveCtx {
    poisson_plan p;
    Sub *s;
    double *scal;  // device scalars of this sub: [0] mean (z pass), [1] sum f, [2] sum r^2, [3] sum fbar^2
};

// forward x (plain or residual input) -> spectrum S
int pass_x_fwd(SolveCtx &c, int prec, const double *f, const double *p, void *S, bool residual,
               bool want_partials)
{
    Sub &s = *c.s;
    const double sb = prec == P_F32 ? 4.0 : 8.0;
    XFwdArgs a{};
    a.f = f;
    a.p = p;
    a.S = S;
    a.tw = s.tab.twx[prec == P_F32 ? 1 : 0]->p;
    a.partials = want_partials ? (double *)s.partials->p : nullptr;
    a.nx = s.d.nx;
    a.ny = s.d.ny;
    a.nz = s.d.nz;
    a.bc_z = s.d.bc_z;
    a.ax = 1.0 / (s.d.dx * s.d.dx);
    a.ay = 1.0 / (s.d.dy * s.d.dy);
    a.az = 1.0 / (s.d.dz * s.d.dz);
    a.sum_f = c.scal + 1;
    a.inv_n = 1.0 / (double)s.N;
    a.residual = residual ? 1 : 0;
    char name[40];
    snprintf(name, sizeof name, residual ? "x_r2c_residual_%s" : "x_r2c_%s", tag(prec));
    const double bytes = (double)s.N * ((residual ? 16.0 : 8.0) + sb);
    int rc = timed(c.p, name, bytes, [&] { return launch_x_fwd(prec, a, nullptr, c.p->stream); });
    if (rc) return rc;
    if (want_partials) {
        // partials hold two interleaved sums per workgroup: plain input ->
        // (sum f, 0) into scal[1..2]; residual -> (sum r^2, sum fbar^2) into scal[2..3]
        double *dst = residual ? c.scal + 2 : c.scal + 1;
        rc = timed(c.p, "sum_partials", (double)s.npart * 16.0, [&] {
            return launch_sum_partials((const double *)s.partials->p, s.npart, 2, dst,
                                       c.p->stream);
        });
    }
    return rc;
}

int pass_y(SolveCtx &c, int prec, void *S, bool inverse)
{
    Sub &s = *c.s;
    if (s.d.ny == 1) return POISSON_OK;  // a length-1 transform is the identity
    YArgs a{S, s.tab.twy[prec == P_F32 ? 1 : 0]->p, s.M, s.d.ny, s.d.nz, inverse ? 1 : 0};
    char name[40];
    snprintf(name, sizeof name, inverse ? "y_inv_%s" : "y_fwd_%s", tag(prec));
    const double bytes = (double)s.N * 2.0 * (prec == P_F32 ? 4.0 : 8.0);
    return timed(c.p, name, bytes, [&] { return launch_y(prec, a, c.p->stream); });
}

int pass_z(SolveCtx &c, int prec, void *S)
{
    Sub &s = *c.s;
    ZArgs a{};
    a.S = S;
    a.tw = s.d.bc_z == POISSON_BC_PERIODIC ? s.tab.twz[prec == P_F32 ? 1 : 0]->p : nullptr;
    a.lamx = (const double *)s.tab.lamx->p;
    a.lamy = (const double *)s.tab.lamy->p;
    a.lamz = (const double *)s.tab.lamz->p;
    a.zero_mean_out = c.scal + 0;
    a.M = s.M;
    a.ny = s.d.ny;
    a.nz = s.d.nz;
    a.nx = s.d.nx;
    a.dz2 = s.d.dz * s.d.dz;
    a.inv_nxny = 1.0 / ((double)s.d.nx * s.d.ny);
    a.inv_ntot = 1.0 / (double)s.N;
    const double bytes = (double)s.N * 2.0 * (prec == P_F32 ? 4.0 : 8.0);
    char name[40];
    if (s.d.bc_z == POISSON_BC_NEUMANN) {
        snprintf(name, sizeof name, "z_walls_%s", tag(prec));
        return timed(c.p, name, bytes, [&] { return launch_z_walls(prec, a, c.p->stream); });
    }
    snprintf(name, sizeof name, "z_periodic_%s", tag(prec));
    return timed(c.p, name, bytes, [&] { return launch_z_periodic(prec, a, c.p->stream); });
}

int pass_x_inv(SolveCtx &c, int prec, const void *S, double *p, bool accumulate)
{
    Sub &s = *c.s;
    XInvArgs a{S, p, s.tab.twx[prec == P_F32 ? 1 : 0]->p, s.d.nx, s.d.ny, s.d.nz,
               accumulate ? 1 : 0};
    char name[40];
    snprintf(name, sizeof name, accumulate ? "x_c2r_accumulate_%s" : "x_c2r_%s", tag(prec));
    const double sb = prec == P_F32 ? 4.0 : 8.0;
    const double bytes = (double)s.N * (sb + (accumulate ? 16.0 : 8.0));
    return timed(c.p, name, bytes, [&] { return launch_x_inv(prec, a, c.p->stream); });
}

// the five passes: S <- transform(f or residual); z solve; p <- (or +=) inverse
int solve_passes(SolveCtx &c, int prec, const double *f, double *p, void *S, bool residual,
                 bool accumulate, bool want_partials)
{
    int rc;
    if ((rc = pass_x_fwd(c, prec, f, p, S, residual, want_partials))) return rc;
    if ((rc = pass_y(c, prec, S, false))) return rc;
    if ((rc = pass_z(c, prec, S))) return rc;
    if ((rc = pass_y(c, prec, S, true))) return rc;
    if ((rc = pass_x_inv(c, prec, S, p, accumulate))) return rc;
    return POISSON_OK;
}

int read_scalars(poisson_plan p, const double *dev, int n, double *host)
{
    hipError_t e = hipMemcpyAsync(host, dev, n * sizeof(double), hipMemcpyDeviceToHost,
                                  p->stream);
    if (e != hipSuccess) return hip_fail("scalar read-back", (int)e);
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail("stream synchronize", (int)e);
    return POISSON_OK;
}

int solve_one(poisson_plan p, int idx, const double *rhs, double *sol, poisson_stats_t *st)
{
    Sub &s = p->subs[idx];
    double *scal = (double *)p->scalars->p + 4 * idx;
    double *hs = p->host_scalars + 4 * idx;
    SolveCtx c{p, &s, scal};
    poisson_stats_t out{0, -1.0, 0.0, POISSON_OK};
    int rc = POISSON_OK;
    const int prec = p->precision;
    if (prec == POISSON_FP64) {
        // the spectrum lives in the solution array (same byte size)
        rc = solve_passes(c, P_F64, rhs, sol, sol, false, false, false);
        if (!rc && st) {
            rc = read_scalars(p, scal, 1, hs);
            out.rhs_mean = hs[0];
        }
    } else if (prec == POISSON_FP32) {
        rc = solve_passes(c, P_F32, rhs, sol, s.S32->p, false, false, true);
        if (!rc && st) {
            rc = read_scalars(p, scal, 2, hs);
            out.rhs_mean = hs[1] / (double)s.N;
        }
    } else {
        // FP32 solve, then r = (f - mean f) - L p in FP64 and p += FP32 solve(r)
        rc = solve_passes(c, P_F32, rhs, sol, s.S32->p, false, false, true);
        double rho_prev = -1.0;
        int corrections = 0;
        for (int it = 0; !rc; ++it) {
            if ((rc = pass_x_fwd(c, P_F32, rhs, sol, s.S32->p, true, true))) break;
            if ((rc = read_scalars(p, scal, 4, hs))) break;
            const double rho = hs[3] > 0 ? std::sqrt(hs[2] / hs[3]) : std::sqrt(hs[2]);
            out.rel_residual = rho;
            out.rhs_mean = hs[1] / (double)s.N;
            if (!std::isfinite(rho)) { rc = POISSON_ERR_NONFINITE; break; }
            if (rho <= p->rtol) break;
            if (corrections >= p->max_refine || (rho_prev >= 0 && rho > 0.5 * rho_prev)) {
                rc = POISSON_ERR_NOT_CONVERGED;
                break;
            }
            rho_prev = rho;
            if ((rc = pass_y(c, P_F32, s.S32->p, false))) break;
            if ((rc = pass_z(c, P_F32, s.S32->p))) break;
            if ((rc = pass_y(c, P_F32, s.S32->p, true))) break;
            if ((rc = pass_x_inv(c, P_F32, s.S32->p, sol, true))) break;
            ++corrections;
        }
        out.iterations = corrections;
    }
    out.status = rc;
    if (st) *st = out;
    return rc;
}

bool overlaps(const double *a, const double *b, long long n)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b, len = (uintptr_t)(n * 8);
    return x < y + len && y < x + len;
}

int create_plan(const poisson_desc_t *descs, int count, void *stream, poisson_plan *out)
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
    if (hipGetDevice(&p->device) != hipSuccess) return POISSON_ERR_HIP;
    std::map<std::string, Tables> cache;
    p->subs.resize(count);
    for (int i = 0; i < count; ++i) {
        poisson_desc_t d = descs[i];
        d.precision = p->precision;
        d.rtol = p->rtol;
        d.max_refine = p->max_refine;
        int rc = build_sub(p->subs[i], d, cache);
        if (rc) return rc;
    }
    int rc = dev_alloc(p->scalars, 4 * sizeof(double) * count);
    if (rc) return rc;
    if (hipMemset(p->scalars->p, 0, 4 * sizeof(double) * count) != hipSuccess)
        return POISSON_ERR_HIP;
    if (hipHostMalloc((void **)&p->host_scalars, 4 * sizeof(double) * count, 0) != hipSuccess) {
        p->host_scalars = nullptr;
        return POISSON_ERR_OUT_OF_MEMORY;
    }
    *out = p.release();
    return POISSON_OK;
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
    return create_plan(d, 1, stream, out);
}

int poisson_batch_plan_create(const poisson_desc_t *descs, int count, void *stream,
                              poisson_plan *out)
{
    return create_plan(descs, count, stream, out);
}

int poisson_solve(poisson_plan plan, const double *rhs, double *sol, poisson_stats_t *stats)
{
    if (!plan || !rhs || !sol) return POISSON_ERR_INVALID_ARG;
    if (plan->subs.size() != 1) return POISSON_ERR_INVALID_ARG;
    if (overlaps(rhs, sol, plan->subs[0].N)) return POISSON_ERR_INVALID_ARG;
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != plan->device) (void)hipSetDevice(plan->device);
    int rc = solve_one(plan, 0, rhs, sol, stats);
    if (cur >= 0 && cur != plan->device) (void)hipSetDevice(cur);
    return rc;
}

int poisson_batch_solve(poisson_plan plan, const double *const *rhs, double *const *sol,
                        poisson_stats_t *stats)
{
    if (!plan || !rhs || !sol) return POISSON_ERR_INVALID_ARG;
    const int n = (int)plan->subs.size();
    for (int i = 0; i < n; ++i) {
        if (!rhs[i] || !sol[i]) return POISSON_ERR_INVALID_ARG;
        if (overlaps(rhs[i], sol[i], plan->subs[i].N)) return POISSON_ERR_INVALID_ARG;
    }
    int first = POISSON_OK;
    for (int i = 0; i < n; ++i) {
        int rc = solve_one(plan, i, rhs[i], sol[i], stats ? &stats[i] : nullptr);
        if (rc && !first) first = rc;
        if (rc == POISSON_ERR_HIP) break;
    }
    return first;
}

int poisson_destroy(poisson_plan plan)
{
    if (!plan) return POISSON_OK;
    (void)hipStreamSynchronize(plan->stream);
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
