// C ABI of the lbm3 library (declared in include/lbm3.h): parameter
// resolution, workspace layout, and the host side of init / step / observe.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm3.h"
#include "lbm3_internal.h"
#include "lbm3_batch.h"
#include "lbm3_params.h"

using lbm3k::Buffers;
using lbm3k::KParams;

struct lbm3 {
    lbm3_params p;
    lbm3_derived d;
    KParams kp;
    Buffers b;
    int prec;
    hipStream_t stream;
    int pc, fc;            // current population buffer, fields it is encoded with
    bool gimp;             // g[pc] not written: the last collision stored (a, phi, v) in b.gp
    bool gmat;             // with gimp: g[pc] holds the implicit g written out (for readers of g)
    bool inited;
    int64_t step;
    std::string err;
};

static std::string g_create_err;

namespace {

const double PI = 3.14159265358979323846;

struct Layout {
    size_t f[2], g[2], rho[2], phi[2], fmu, gp, scratch, counters, partials, result, total;
};

int lattice_D(int32_t lattice) { return lattice == LBM3_D2Q9 ? 2 : (lattice == LBM3_D3Q27 ? 3 : 0); }

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool validate(const lbm3_params *p, std::string &why)
{
    if (!p) { why = "null parameters"; return false; }
    int D = lattice_D(p->lattice);
    if (!D) { why = "lattice must be 9 (D2Q9) or 27 (D3Q27)"; return false; }
    int nz = D == 2 ? 1 : p->n[2];
    if (p->n[0] < 1 || p->n[1] < 1 || nz < 1) { why = "grid extents must be positive"; return false; }
    if (D == 2 && p->n[2] > 1) { why = "n[2] must be 1 for D2Q9"; return false; }
    int nw = D == 2 ? p->n[1] : nz;
    if (p->walls && nw < 3) { why = "the wall axis needs at least 3 layers"; return false; }
    // node offsets inside one population array are 32-bit in the kernels
    if ((long long)p->n[0] * p->n[1] * nz >= (1LL << 32)) { why = "grid too large (2^32 nodes or more)"; return false; }
    // and so are the byte offsets inside one population or field array
    if ((long long)p->n[0] * p->n[1] * nz * (p->precision == LBM3_FP64 ? 8 : 4) >= (1LL << 32)) {
        why = "grid too large (one population array of 4 GiB or more)";
        return false;
    }
    if (!(p->rho_l > 0.0) || !(p->rho_g > 0.0) || !(p->rho_l > p->rho_g)) {
        why = "need rho_l > rho_g > 0";
        return false;
    }
    if (!(p->chi > 0.0)) { why = "chi must be positive"; return false; }
    if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5)) { why = "relaxation times must exceed 1/2"; return false; }
    if (p->wetting < 0 || p->wetting > 2) { why = "unknown wetting method"; return false; }
    if (p->precision < 0 || p->precision > 2) { why = "unknown precision"; return false; }
    if (p->walls && p->wetting != LBM3_WET_FORCE) {
        for (int w = 0; w < 2; ++w)
            for (int k = 0; k < 3; ++k) {
                double t = p->theta_deg[w][k];
                if (!(t > 0.0 && t < 180.0)) { why = "contact angles must lie in (0, 180)"; return false; }
                double ct = std::cos(t * PI / 180.0) / std::sin(t * PI / 180.0);
                if (std::fabs(ct) > 3.0 + 1e-9 && p->wetting == LBM3_WET_GEOM_INTERP) {
                    why = "geometric interpolation supports |cot(theta)| <= 3 (theta in [18.43, 161.57] deg)";
                    return false;
                }
            }
    }
    if (p->native == 0) {
        if (!(p->gamma12 > 0 && p->gamma13 > 0 && p->gamma23 > 0 && p->width > 0)) {
            why = "native = 0 needs positive gamma12, gamma13, gamma23 and width";
            return false;
        }
    }
    return true;
}

// the alpha-statistics slots: kCntSlots shared ones, then one per block of
// the small 2D fused kernel
size_t counter_slots(const lbm3_params *p)
{
    const int D = lattice_D(p->lattice);
    return (size_t)lbm3k::kCntSlots + (size_t)lbm3k::small2d_block_slots(D, p->n[0], p->n[D - 1]);
}

// tau_g = 1 with collisions in the 3D two-kernel step: the post-collision g
// is g^eq of (a, phi, v), Eqs. 33-35, so the collision stores those five
// values per node in the compute type (20 bytes, 40 in FP64) instead of
// pushing 27 populations, and the next moments pass rebuilds the delivered
// g from them (with FP16 storage g is then never rounded to FP16)
bool implicit_g(const lbm3_params *p)
{
    return p->lattice == LBM3_D3Q27 && p->tau_g == 1.0 &&
           !(p->flags & (LBM3_NO_COLLIDE | LBM3_FUSED_3D | LBM3_STORED_G));
}

Layout layout(const lbm3_params *p)
{
    Layout L{};
    int D = lattice_D(p->lattice);
    int Q = D == 2 ? 9 : 27;
    long long N = (long long)p->n[0] * p->n[1] * (D == 2 ? 1 : p->n[2]);
    // every array of a block QS elements after the previous one, every field QS long
    const long long QS = lbm3k::array_stride(N);
    size_t s = p->precision == LBM3_FP64 ? 8 : (p->precision == LBM3_FP32 ? 4 : 2);
    size_t r = p->precision == LBM3_FP64 ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    for (int k = 0; k < 2; ++k) L.f[k] = take((size_t)Q * QS * s);
    // implicit g: nothing writes a second g set (the collision stores the
    // five g^eq values; g is written only by the initialisation and by
    // exports, each into the current set), so both parities share one
    if (implicit_g(p)) L.g[0] = L.g[1] = take((size_t)Q * QS * s);
    else
        for (int k = 0; k < 2; ++k) L.g[k] = take((size_t)Q * QS * s);
    for (int k = 0; k < 2; ++k) L.rho[k] = take((size_t)QS * r);
    for (int k = 0; k < 2; ++k) L.phi[k] = take((size_t)QS * r);
    L.fmu = D == 3 ? take((size_t)(D + 1) * QS * r) : 0;  // F, mu_phi of the two-kernel step
    L.gp = implicit_g(p) ? take((size_t)5 * QS * r) : 0;    // (a, phi, v) of g^eq
    L.scratch = take((size_t)N * 8);
    L.counters = take(counter_slots(p) * lbm3k::kCntStride * sizeof(unsigned long long));
    L.partials = take((size_t)1024 * 16 * sizeof(double));
    L.result = take(32 * sizeof(double));
    L.total = off;
    return L;
}

double cot_deg(double deg)
{
    double t = deg * PI / 180.0;
    double c = std::cos(t) / std::sin(t);
    double r = std::nearbyint(c);
    if (std::fabs(c - r) < 1e-9) c = r;  // exact lattice copies at the special angles
    return c;
}

lbm3_status set_err(lbm3 *h, lbm3_status st, const std::string &m)
{
    if (h) h->err = m;
    else g_create_err = m;
    return st;
}

lbm3_status hip_err(lbm3 *h, hipError_t e, const char *where)
{
    return set_err(h, LBM3_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t lbm3_footprint(const lbm3_params *p)
{
    std::string why;
    if (!validate(p, why)) return 0;
    return layout(p).total;
}

lbm3_status lbm3_resolve(const lbm3_params *p, lbm3_derived *out)
{
    std::string why;
    if (!out || !validate(p, why)) return LBM3_EINVAL;
    lbm3_derived d{};
    if (!lbm3h::coexistence(p->rho_l / p->rho_g, p->rho_l, d.a, d.b, d.T, d.C, d.psi0, d.rho_l, d.rho_g))
        return LBM3_EINVAL;
    if (p->native) {
        for (int k = 0; k < 3; ++k) { d.lambda[k] = p->lambda[k]; d.kappa[k] = p->kappa[k]; }
    } else {
        if (lbm3h::calibrate(p->gamma12, p->gamma13, p->gamma23, p->width, d.rho_l, d.rho_g, p->chi, d.a,
                             d.b, d.T, d.C, d.psi0, d.lambda, d.kappa) != 0)
            return LBM3_ECALIB;
    }
    double drho = d.rho_l - d.rho_g;
    d.kappa_rr = d.kappa[0] + (d.kappa[1] + d.kappa[2]) / (4.0 * drho * drho);
    d.kappa_pp = (d.kappa[1] + d.kappa[2]) / (4.0 * p->chi * p->chi);
    d.kappa_x = (d.kappa[1] - d.kappa[2]) / (4.0 * p->chi * drho);
    d.beta = 1.0 / (2.0 * p->tau_f);
    for (int w = 0; w < 2; ++w)
        for (int k = 0; k < 3; ++k) d.cot_theta[w][k] = p->walls ? cot_deg(p->theta_deg[w][k]) : 0.0;
    *out = d;
    return LBM3_OK;
}

lbm3_status lbm3_create(const lbm3_params *p, void *ws, size_t bytes, void *stream, lbm3 **out)
{
    std::string why;
    if (!out) return set_err(nullptr, LBM3_EINVAL, "null output handle");
    *out = nullptr;
    if (!validate(p, why)) return set_err(nullptr, LBM3_EINVAL, why);
    Layout L = layout(p);
    if (!ws || bytes < L.total) return set_err(nullptr, LBM3_ENOMEM, "workspace smaller than lbm3_footprint()");
    if (((uintptr_t)ws & 255) != 0) return set_err(nullptr, LBM3_EINVAL, "workspace must be 256-byte aligned");
    lbm3_derived d;
    lbm3_status st = lbm3_resolve(p, &d);
    if (st != LBM3_OK)
        return set_err(nullptr, st, st == LBM3_ECALIB ? "tension calibration failed" : "no Carnahan-Starling coexistence for rho_l/rho_g");
    lbm3 *h = new (std::nothrow) lbm3();
    if (!h) return set_err(nullptr, LBM3_ENOMEM, "host allocation failed");
    h->p = *p;
    h->d = d;
    h->prec = p->precision;
    h->stream = (hipStream_t)stream;
    int D = lattice_D(p->lattice);
    KParams &k = h->kp;
    k.D = D;
    k.Q = D == 2 ? 9 : 27;
    k.nx = p->n[0];
    k.ny = p->n[1];
    k.nz = D == 2 ? 1 : p->n[2];
    k.nw = D == 2 ? k.ny : k.nz;
    k.walls = p->walls ? 1 : 0;
    k.N = (long long)k.nx * k.ny * k.nz;
    k.QS = lbm3k::array_stride(k.N);
    k.PS = D == 2 ? k.nx : (long long)k.nx * k.ny;
    k.rho_l = d.rho_l;
    k.rho_g = d.rho_g;
    k.drho = d.rho_l - d.rho_g;
    k.chi = p->chi;
    k.a = d.a; k.b = d.b; k.T = d.T; k.C = d.C; k.psi0 = d.psi0;
    k.lam1 = d.lambda[0]; k.lam2 = d.lambda[1]; k.lam3 = d.lambda[2];
    k.krr = d.kappa_rr; k.kpp = d.kappa_pp; k.kx = d.kappa_x;
    k.beta = d.beta;
    k.inv_tau_g = 1.0 / p->tau_g;
    k.Gamma = p->Gamma;
    k.wetting = p->wetting;
    for (int w = 0; w < 2; ++w) {
        for (int c = 0; c < 3; ++c) k.cot[w][c] = d.cot_theta[w][c];
        for (int c = 0; c < 2; ++c) k.kw[w][c] = p->kw[w][c];
    }
    // below this deviation alpha comes from the expansion of the entropy
    // equation; FP32 keeps Newton to deviations where its root is resolved
    k.alpha_eps = p->alpha_eps > 0 ? p->alpha_eps : (p->precision == LBM3_FP64 ? 1e-3 : 1e-2);
    k.alpha_tol = p->alpha_tol > 0 ? p->alpha_tol : (p->precision == LBM3_FP64 ? 1e-10 : 1e-5);
    k.alpha_maxit = p->alpha_maxit > 0 ? p->alpha_maxit : 20;
    k.detect_ratio = p->detect_ratio > 0 ? p->detect_ratio : 0.01;
    k.flags = p->flags;
    char *base = (char *)ws;
    Buffers &b = h->b;
    for (int i = 0; i < 2; ++i) {
        b.f[i] = base + L.f[i];
        b.g[i] = base + L.g[i];
        b.rho[i] = base + L.rho[i];
        b.phi[i] = base + L.phi[i];
    }
    b.fmu = D == 3 ? (void *)(base + L.fmu) : nullptr;
    b.gp = L.gp ? (void *)(base + L.gp) : nullptr;
    b.scratch = (double *)(base + L.scratch);
    b.counters = (unsigned long long *)(base + L.counters);
    b.partials = (double *)(base + L.partials);
    b.result = (double *)(base + L.result);
    b.n_partials = 1024;
    h->pc = h->fc = 0;
    h->gimp = h->gmat = false;
    h->inited = false;
    h->step = 0;
    *out = h;
    return LBM3_OK;
}

lbm3_status lbm3_init(lbm3 *h, const double *rho0, const double *phi0)
{
    if (!h) return LBM3_EINVAL;
    if (!rho0 || !phi0) return set_err(h, LBM3_EINVAL, "null initial field");
    const KParams &k = h->kp;
    size_t bytes = (size_t)k.N * sizeof(double);
    for (long long n = 0; n < k.N; ++n) {
        long long p = k.D == 2 ? n / k.nx : n / ((long long)k.nx * k.ny);
        bool fluid = !k.walls || (p >= 1 && p <= k.nw - 2);
        if (fluid && !(rho0[n] > 0.0 && std::isfinite(rho0[n]) && std::isfinite(phi0[n])))
            return set_err(h, LBM3_EINVAL, "initial rho must be positive and finite on fluid nodes");
    }
    hipError_t e;
    // populations of the ghost layers are never read by a step; zeroing both
    // buffers keeps exported arrays deterministic
    size_t pop_bytes = (size_t)k.Q * k.QS * (h->prec == LBM3_FP64 ? 8 : (h->prec == LBM3_FP32 ? 4 : 2));
    for (int i = 0; i < 2; ++i)
        if ((e = hipMemsetAsync(h->b.f[i], 0, pop_bytes, h->stream)) != hipSuccess ||
            (e = hipMemsetAsync(h->b.g[i], 0, pop_bytes, h->stream)) != hipSuccess)
            return hip_err(h, e, "clear populations");
    const double *src[2] = {rho0, phi0};
    for (int which = 0; which < 2; ++which) {
        if ((e = hipMemcpyAsync(h->b.scratch, src[which], bytes, hipMemcpyHostToDevice, h->stream)) != hipSuccess)
            return hip_err(h, e, "upload");
        if (lbm3k::launch_init_field(k, h->prec, h->b, which, h->stream)) return set_err(h, LBM3_EDEVICE, "init launch failed");
    }
    if (lbm3k::launch_ghost(k, h->prec, h->b, 0, h->stream)) return set_err(h, LBM3_EDEVICE, "ghost launch failed");
    if (lbm3k::launch_init(k, h->prec, h->b, h->stream)) return set_err(h, LBM3_EDEVICE, "init launch failed");
    if ((e = hipMemsetAsync(h->b.counters, 0, counter_slots(&h->p) * lbm3k::kCntStride * sizeof(unsigned long long),
                            h->stream)) != hipSuccess)
        return hip_err(h, e, "counters");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "init");
    h->pc = h->fc = 0;
    h->gimp = h->gmat = false;  // the populations just written are stored, g included
    h->step = 0;
    h->inited = true;
    return LBM3_OK;
}

// The launches of one step: moments, ghost layers (unless the fused kernel
// fills them itself), then the fused update.
static int launch_moments(lbm3 *h)
{
    return h->gimp ? lbm3k::launch_moments_imp(h->kp, h->prec, h->b, h->pc, h->fc, h->stream)
                   : lbm3k::launch_moments(h->kp, h->prec, h->b, h->pc, h->fc, h->stream);
}

// g[pc] written out where something reads the stored g.  The state stays
// implicit: the next moments pass still rebuilds g from the five values
// (with FP16 storage the written copy is rounded, the five values are not).
static int materialize_g(lbm3 *h, hipStream_t st)
{
    if (!h->gimp || h->gmat) return 0;
    if (lbm3k::launch_g_materialize(h->kp, h->prec, h->b, h->pc, h->fc, st)) return -1;
    h->gmat = true;
    return 0;
}

// after the collision of a step: whether it stored (a, phi, v) instead of g
static void stepped(lbm3 *h)
{
    h->pc ^= 1;
    h->fc ^= 1;
    h->step++;
    h->gimp = h->b.gp != nullptr;
    h->gmat = false;
}

static int launch_step(lbm3 *h, int which)
{
    const KParams &k = h->kp;
    switch (which) {
    case 0: return launch_moments(h);
    case 1: return lbm3k::fused_fills_ghost(k) ? 0 : lbm3k::launch_ghost(k, h->prec, h->b, 1 - h->fc, h->stream);
    default: return lbm3k::launch_fused(k, h->prec, h->b, h->pc, h->fc, h->stream);
    }
}

lbm3_status lbm3_step(lbm3 *h, int64_t nsteps)
{
    if (!h) return LBM3_EINVAL;
    if (!h->inited) return set_err(h, LBM3_ESTATE, "step before init");
    if (nsteps < 0) return set_err(h, LBM3_EINVAL, "negative step count");
    for (int64_t t = 0; t < nsteps; ++t) {
        if (launch_step(h, 0) || launch_step(h, 1) || launch_step(h, 2))
            return set_err(h, LBM3_EDEVICE, "kernel launch failed");
        stepped(h);
    }
    return LBM3_OK;
}

lbm3_status lbm3_step_profiled(lbm3 *h, int64_t nsteps, int32_t sample_every, double *kernel_ms)
{
    if (!h) return LBM3_EINVAL;
    if (!h->inited) return set_err(h, LBM3_ESTATE, "step before init");
    if (nsteps < 0 || sample_every < 1) return set_err(h, LBM3_EINVAL, "bad step count or sampling stride");
    // per sampled step a start and a stop event for each of the three stages,
    // recorded by the stage's own kernels (no marker packets between them),
    // and in a two-kernel last stage the end of its first kernel and the
    // start of its second
    constexpr int PER = 8;
    const int batch = 64;  // sampled steps between host synchronisations
    hipEvent_t ev[PER * batch], first = nullptr, last = nullptr;
    int made = 0;
    hipError_t e = hipSuccess;
    lbm3_status st = LBM3_OK;
    double acc[5] = {0, 0, 0, 0, 0}, span = 0;
    int64_t sampled = 0;
    const bool no_ghost = lbm3k::fused_fills_ghost(h->kp);
    const bool split = lbm3k::two_kernel_step(h->kp);
    for (; made < PER * batch; ++made)
        if ((e = hipEventCreate(&ev[made])) != hipSuccess) break;
    if (e == hipSuccess) e = hipEventCreate(&first);
    if (e == hipSuccess) e = hipEventCreate(&last);
    if (e == hipSuccess) e = hipEventRecord(first, h->stream);
    if (e != hipSuccess) st = hip_err(h, e, "event setup");
    int pending = 0;  // sampled steps whose events are not yet read
    auto elapsed = [&](hipEvent_t a, hipEvent_t b, double &sum) -> bool {
        float ms = 0;
        if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) return false;
        sum += ms;
        return true;
    };
    auto drain = [&]() -> bool {
        if (!pending) return true;
        if ((e = hipEventSynchronize(ev[PER * (pending - 1) + 5])) != hipSuccess) return false;
        for (int s = 0; s < pending; ++s) {
            hipEvent_t *E = ev + PER * s;
            for (int j = 0; j < 3; ++j) {
                if (j == 1 && no_ghost) continue;
                if (!elapsed(E[2 * j], E[2 * j + 1], acc[j])) return false;
            }
            if (split && (!elapsed(E[4], E[6], acc[3]) || !elapsed(E[7], E[5], acc[4]))) return false;
        }
        sampled += pending;
        pending = 0;
        return true;
    };
    for (int64_t t = 0; t < nsteps && st == LBM3_OK; ++t) {
        const bool timed = t % sample_every == 0;
        hipEvent_t *E = ev + PER * pending;
        int r = 0;
        for (int j = 0; j < 3 && !r; ++j) {
            if (j == 1 && no_ghost) continue;
            if (timed) lbm3k::set_stage_events(E[2 * j], E[2 * j + 1], j == 2 && split ? E[6] : nullptr,
                                               j == 2 && split ? E[7] : nullptr);
            r = launch_step(h, j);
            lbm3k::set_stage_events(nullptr, nullptr, nullptr, nullptr);
        }
        if (r) { st = set_err(h, LBM3_EDEVICE, "kernel launch failed"); break; }
        stepped(h);
        if (timed && ++pending == batch && !drain()) st = hip_err(h, e, "profiled step");
    }
    if (st == LBM3_OK && !drain()) st = hip_err(h, e, "profiled step");
    if (st == LBM3_OK) {
        float ms = 0;
        if ((e = hipEventRecord(last, h->stream)) != hipSuccess || (e = hipEventSynchronize(last)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, first, last)) != hipSuccess)
            st = hip_err(h, e, "profiled span");
        span = ms;
    }
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(ev[i]);
    if (first) (void)hipEventDestroy(first);
    if (last) (void)hipEventDestroy(last);
    if (kernel_ms) {
        for (int j = 0; j < 3; ++j) kernel_ms[j] = sampled ? acc[j] / (double)sampled : 0.0;
        kernel_ms[3] = span;
        kernel_ms[4] = (double)sampled;
        kernel_ms[5] = sampled ? acc[3] / (double)sampled : 0.0;
        kernel_ms[6] = sampled ? acc[4] / (double)sampled : 0.0;
        kernel_ms[7] = 0.0;
    }
    return st;
}

lbm3_status lbm3_observe(lbm3 *h, uint32_t what, lbm3_obs *out, double *rho_out, double *phi_out, double *f_out,
                         double *g_out)
{
    if (!h) return LBM3_EINVAL;
    if (!h->inited) return set_err(h, LBM3_ESTATE, "observe before init");
    const KParams &k = h->kp;
    hipError_t e;
    size_t bytes = (size_t)k.N * sizeof(double);
    lbm3_status status = LBM3_OK;
    if ((what & (LBM3_OBS_POPS | LBM3_OBS_SUMS)) && materialize_g(h, h->stream))
        return set_err(h, LBM3_EDEVICE, "kernel launch failed");
    if (what & LBM3_OBS_FIELDS) {
        // moments and ghost layers of the current state into the spare fields
        if (launch_moments(h) ||
            lbm3k::launch_ghost(k, h->prec, h->b, 1 - h->fc, h->stream))
            return set_err(h, LBM3_EDEVICE, "kernel launch failed");
        double *dst[2] = {rho_out, phi_out};
        for (int which = 0; which < 2; ++which) {
            if (!dst[which]) continue;
            if (lbm3k::launch_export_field(k, h->prec, h->b, 1 - h->fc, which, h->stream))
                return set_err(h, LBM3_EDEVICE, "export launch failed");
            if ((e = hipMemcpyAsync(dst[which], h->b.scratch, bytes, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
                return hip_err(h, e, "download");
            if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "download");
        }
    }
    if (what & LBM3_OBS_POPS) {
        double *dst[2] = {f_out, g_out};
        for (int which = 0; which < 2; ++which) {
            if (!dst[which]) continue;
            for (int i = 0; i < k.Q; ++i) {
                if (lbm3k::launch_export_pop(k, h->prec, h->b, h->pc, h->fc, which, i, h->stream))
                    return set_err(h, LBM3_EDEVICE, "export launch failed");
                if ((e = hipMemcpyAsync(dst[which] + (size_t)i * k.N, h->b.scratch, bytes, hipMemcpyDeviceToHost,
                                        h->stream)) != hipSuccess)
                    return hip_err(h, e, "download");
                if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "download");
            }
        }
    }
    if (what & LBM3_OBS_SUMS) {
        if (!out) return set_err(h, LBM3_EINVAL, "null observable output");
        if (lbm3k::launch_observe(k, h->prec, h->b, h->pc, h->fc, h->stream))
            return set_err(h, LBM3_EDEVICE, "observe launch failed");
        double r[16];
        const size_t nslots = counter_slots(&h->p);
        std::vector<unsigned long long> slots(nslots * lbm3k::kCntStride);
        if ((e = hipMemcpyAsync(r, h->b.result, sizeof(r), hipMemcpyDeviceToHost, h->stream)) != hipSuccess ||
            (e = hipMemcpyAsync(slots.data(), h->b.counters, slots.size() * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
            return hip_err(h, e, "observe download");
        if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "observe");
        unsigned long long c[4] = {0, 0, 0, 0};
        for (size_t k = 0; k < nslots; ++k)
            for (int q = 0; q < 4; ++q) c[q] += slots[k * lbm3k::kCntStride + q];
        for (int q = 0; q < 3; ++q) out->mass[q] = r[q];
        out->rho_sum = r[3];
        out->phi_sum = r[4];
        for (int q = 0; q < 3; ++q) out->mom[q] = r[5 + q];
        out->kinetic = r[8];
        out->umax = r[9];
        out->n_bad = (int64_t)r[12];
        out->n_newton = (int64_t)c[0];
        out->n_shortcut = (int64_t)c[1];
        out->n_fallback = (int64_t)c[2];
        out->n_fast = (int64_t)c[3];
        out->step = h->step;
        if (out->n_bad > 0) status = set_err(h, LBM3_EUNSTABLE, "NaN or non-positive density in the state");
        else if (out->n_fast > 0)
            status = set_err(h, LBM3_EUNSTABLE, "a collision had |u + du| >= 1 (the lattice speed)");
    }
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "observe");
    return status;
}

lbm3_status lbm3_contact_angle(lbm3 *h, int32_t comp, int32_t wall, double exclude, double *out)
{
    if (!h) return LBM3_EINVAL;
    if (!h->inited) return set_err(h, LBM3_ESTATE, "contact angle before init");
    if (!out || (comp != 2 && comp != 3) || (wall != 0 && wall != 1) || !h->kp.walls)
        return set_err(h, LBM3_EINVAL, "contact angle needs comp 2 or 3, wall 0 or 1, a walled grid");
    const KParams &k = h->kp;
    hipError_t e;
    if (launch_moments(h) ||
        lbm3k::launch_contour(k, h->prec, h->b, 1 - h->fc, comp, wall, exclude, h->stream))
        return set_err(h, LBM3_EDEVICE, "contour launch failed");
    double r[16];
    if ((e = hipMemcpyAsync(r, h->b.result, sizeof(r), hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
        return hip_err(h, e, "contour download");
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_err(h, e, "contour");
    // normal equations of the Kasa fit, unknowns (D, E, [F,] G)
    int m = k.D == 2 ? 3 : 4;
    double A[4][5];
    int idx = 0;
    for (int a = 0; a < m; ++a)
        for (int bb = a; bb < m; ++bb) { A[a][bb] = A[bb][a] = r[idx++]; }
    for (int a = 0; a < m; ++a) A[a][m] = -r[idx++];
    double npts = A[m - 1][m - 1];
    if (npts < m + 1) return set_err(h, LBM3_EINVAL, "too few contour points for a circle fit");
    for (int c = 0; c < m; ++c) {  // Gaussian elimination with partial pivoting
        int piv = c;
        for (int rr = c + 1; rr < m; ++rr)
            if (std::fabs(A[rr][c]) > std::fabs(A[piv][c])) piv = rr;
        for (int cc = 0; cc <= m; ++cc) std::swap(A[c][cc], A[piv][cc]);
        for (int rr = 0; rr < m; ++rr) {
            if (rr == c) continue;
            double f = A[rr][c] / A[c][c];
            for (int cc = c; cc <= m; ++cc) A[rr][cc] -= f * A[c][cc];
        }
    }
    double sol[4];
    for (int a = 0; a < m; ++a) sol[a] = A[a][m] / A[a][a];
    double cen[3] = {0, 0, 0}, rr2 = 0;
    for (int a = 0; a < m - 1; ++a) { cen[a] = -0.5 * sol[a]; rr2 += cen[a] * cen[a]; }
    double R = std::sqrt(rr2 - sol[m - 1]);
    double wplane = wall == 0 ? 0.5 : k.nw - 1.5;
    double hc = cen[k.D - 1];
    double hgt = wall == 0 ? hc - wplane : wplane - hc;
    double cth = -hgt / R;
    cth = cth > 1 ? 1 : (cth < -1 ? -1 : cth);
    out[0] = std::acos(cth) * 180.0 / PI;
    out[1] = cen[0];
    out[2] = cen[1];
    out[3] = cen[2];
    out[4] = R;
    out[5] = npts;
    return LBM3_OK;
}

lbm3_status lbm3_destroy(lbm3 *h)
{
    if (!h) return LBM3_EINVAL;
    delete h;
    return LBM3_OK;
}

const char *lbm3_last_error(const lbm3 *h)
{
    return h ? h->err.c_str() : g_create_err.c_str();
}

lbm3_status lbm3_batch_workspace(lbm3 *const *hs, int32_t n, size_t *bytes)
{
    if (!bytes) return LBM3_EINVAL;
    *bytes = lbm3b::image_bytes(hs, n);
    return *bytes ? LBM3_OK : LBM3_EINVAL;
}

lbm3_status lbm3_step_batch(lbm3 *const *hs, int32_t n, int64_t nsteps, void *stream, void *ws, size_t ws_bytes)
{
    if (nsteps < 0) return LBM3_EINVAL;
    lbm3b::Image img;
    lbm3_status st = lbm3b::build(hs, n, img);
    if (st != LBM3_OK) return st;
    if (!ws || ws_bytes < img.bytes.size() || ((uintptr_t)ws & 255) != 0) return LBM3_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    // the image is in pageable memory: wait for the copy before it goes
    if (hipMemcpyAsync(ws, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBM3_EDEVICE;
    return lbm3b::enqueue(hs, n, img, ws, 0, nsteps, s);
}

}  // extern "C"

// ------------------------------------------- batched stepping, no workspace
// The descriptor image of lbm3_step_batch_static lives in this file-scope
// device array instead of a caller workspace: every device the library runs
// on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy (in host code it is only a stand-in
// for the symbol): the device address comes from hipGetSymbolAddress, once
// per device with that device current, and is kept per device.
namespace {
constexpr size_t kStaticImageBytes = LBM3_STEP_BATCH_STATIC_MAX_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticImageBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

lbm3_status scratch_address(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LBM3_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM3_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LBM3_OK;
}
}  // namespace

extern "C" {

lbm3_status lbm3_step_batch_static(lbm3 *const *hs, int32_t n, int64_t nsteps, void *stream)
{
    if (nsteps < 0) return LBM3_EINVAL;
    lbm3b::Image img;
    lbm3_status st = lbm3b::build(hs, n, img);
    if (st != LBM3_OK) return st;
    if (img.bytes.size() > kStaticImageBytes) {
        for (int i = 0; i < n; ++i)
            hs[i]->err = "batch image of " + std::to_string(img.bytes.size()) + " bytes exceeds the static " +
                         std::to_string(kStaticImageBytes) + "-byte scratch array";
        return LBM3_EINVAL;
    }
    void *dev_img = nullptr;
    if ((st = scratch_address(&dev_img)) != LBM3_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the image is in pageable memory: wait for the copy before it goes
    if (hipMemcpyAsync(dev_img, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return LBM3_EDEVICE;
    return lbm3b::enqueue(hs, n, img, dev_img, 0, nsteps, s);
}

}  // extern "C"

// ------------------------------------------------------------- batching --
namespace lbm3b {

using lbm3k::FusedGeom;
using lbm3k::SimDesc;

static bool check_handles(lbm3 *const *hs, int n)
{
    if (!hs || n < 1) return false;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || !hs[i]->inited) return false;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return false;  // one handle twice would step twice
    }
    return true;
}

// launches of the batch: moments per (D, precision), ghost layers per
// (D, precision) where the step has them, fused (or stencil) per (tile
// class, precision), collide per (D, precision, implicit g or not) for
// two-kernel 3D steps
static void plan(lbm3 *const *hs, int n, std::vector<Launch> &L)
{
    auto find = [&](int kind, int D, int prec, int cls) -> Launch & {
        for (auto &l : L)
            if (l.kind == kind && l.D == D && l.prec == prec && l.cls == cls) return l;
        Launch l;
        l.kind = kind;
        l.D = D;
        l.prec = prec;
        l.cls = cls;
        l.table_off = 0;
        l.prefix.push_back(0);
        L.push_back(l);
        return L.back();
    };
    for (int i = 0; i < n; ++i) {
        const KParams &k = hs[i]->kp;
        int prec = hs[i]->prec;
        Launch &m = find(0, k.D, prec, 0);
        m.sims.push_back(i);
        m.prefix.push_back(m.prefix.back() + lbm3k::moments_batch_blocks(k, prec, hs[i]->b.gp != nullptr));
        long long gb = lbm3k::ghost_blocks(k);
        if (gb > 0) {
            Launch &g = find(1, k.D, prec, 0);
            g.sims.push_back(i);
            g.prefix.push_back(g.prefix.back() + gb);
        }
        FusedGeom fg = lbm3k::fused_geometry(k, prec);
        Launch &f = find(2, k.D, prec, fg.cls);
        f.sims.push_back(i);
        f.prefix.push_back(f.prefix.back() + (long long)fg.ntiles * fg.nchunks);
        long long cb = lbm3k::collide_blocks(k);
        if (cb > 0) {
            // simulations with implicit g apart from the others (class 1)
            Launch &c = find(3, k.D, prec, hs[i]->b.gp ? 1 : 0);
            c.sims.push_back(i);
            c.prefix.push_back(c.prefix.back() + cb);
        }
    }
    // kernel classes in step order
    std::stable_sort(L.begin(), L.end(), [](const Launch &a, const Launch &b) { return a.kind < b.kind; });
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t image_bytes(lbm3 *const *hs, int n)
{
    if (!check_handles(hs, n)) return 0;
    std::vector<Launch> L;
    plan(hs, n, L);
    size_t bytes = align256(sizeof(SimDesc) * (size_t)n);
    for (auto &l : L) bytes += align256(sizeof(int) * (size_t)l.prefix.back());
    return bytes;
}

lbm3_status build(lbm3 *const *hs, int n, Image &img)
{
    if (!check_handles(hs, n)) return LBM3_EINVAL;
    img.launches.clear();
    plan(hs, n, img.launches);
    img.desc_bytes = align256(sizeof(SimDesc) * (size_t)n);
    size_t off = img.desc_bytes;
    for (auto &l : img.launches) {
        l.table_off = off;
        off += align256(sizeof(int) * (size_t)l.prefix.back());
    }
    img.bytes.assign(off, 0);
    SimDesc *d = (SimDesc *)img.bytes.data();
    for (int i = 0; i < n; ++i) {
        const lbm3 *h = hs[i];
        SimDesc &s = d[i];
        s.kp = h->kp;
        for (int j = 0; j < 2; ++j) {
            s.f[j] = h->b.f[j];
            s.g[j] = h->b.g[j];
            s.rho[j] = h->b.rho[j];
            s.phi[j] = h->b.phi[j];
        }
        s.fmu = h->b.fmu;
        s.gp = h->b.gp;
        s.gimp0 = h->gimp ? 1 : 0;
        s.mchunk = h->kp.D == 3 ? lbm3k::moments_march_chunk(h->kp) : 0;
        s.counters = h->b.counters;
        s.pc = h->pc;
        s.fc = h->fc;
        FusedGeom fg = lbm3k::fused_geometry(h->kp, h->prec);
        s.chunk = fg.chunk;
        s.ntiles = fg.ntiles;
        s.fblk0 = s.mblk0 = s.gblk0 = s.cblk0 = 0;
    }
    for (auto &l : img.launches) {
        int *t = (int *)(img.bytes.data() + l.table_off);
        for (size_t k = 0; k < l.sims.size(); ++k) {
            int i = l.sims[k];
            long long b0 = l.prefix[k], b1 = l.prefix[k + 1];
            if (b1 > (long long)INT32_MAX) return LBM3_EINVAL;
            (l.kind == 0 ? d[i].mblk0 : l.kind == 1 ? d[i].gblk0 : l.kind == 2 ? d[i].fblk0 : d[i].cblk0) = (int)b0;
            for (long long b = b0; b < b1; ++b) t[b] = i;
        }
    }
    return LBM3_OK;
}

lbm3_status enqueue(lbm3 *const *hs, int m, const Image &img, const void *dev_base, int64_t phase0, int64_t steps,
                    hipStream_t stream)
{
    if (m < 1 || steps < 0) return LBM3_EINVAL;
    const SimDesc *d = (const SimDesc *)dev_base;
    const char *base = (const char *)dev_base;
    for (int64_t t = 0; t < steps; ++t) {
        const int phase = (int)((phase0 + t) & 1);
        for (const auto &l : img.launches) {
            // blocks of the simulations among the first m
            size_t k = 0;
            while (k < l.sims.size() && l.sims[k] < m) ++k;
            long long nb = l.prefix[k];
            if (nb == 0) continue;
            const int *tab = (const int *)(base + l.table_off);
            const bool first = phase0 + t == 0;
            int r = l.kind == 0 ? lbm3k::launch_moments_batch(l.D, l.prec, d, tab, nb, phase, first, stream)
                  : l.kind == 1 ? lbm3k::launch_ghost_batch(l.D, l.prec, d, tab, nb, phase, stream)
                  : l.kind == 2 ? lbm3k::launch_fused_batch(l.cls, l.prec, d, tab, nb, phase, stream)
                                : lbm3k::launch_collide_batch(l.D, l.prec, l.cls == 1, d, tab, nb, phase, stream);
            if (r) return LBM3_EDEVICE;
        }
    }
    for (int i = 0; i < m; ++i) {
        if (steps & 1) {
            hs[i]->pc ^= 1;
            hs[i]->fc ^= 1;
        }
        hs[i]->step += steps;
        if (steps > 0 && hs[i]->b.gp) {
            hs[i]->gimp = true;
            hs[i]->gmat = false;
        }
    }
    return LBM3_OK;
}

}  // namespace lbm3b
