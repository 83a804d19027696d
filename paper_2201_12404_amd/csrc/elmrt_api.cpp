// elmrt_api.cpp -- C ABI of the library (declared in include/elmrt.h): parameter
// validation, workspace carving, the Peng-Robinson host thermodynamics, and
// the enqueueing of the kernels of elmrt_kernels.hip on the caller's stream.
#include "../../include/elmrt.h"
#include "elmrt_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <vector>

namespace {

thread_local std::string g_last_error;

elmrt_status fail(elmrt_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace

void elmrt::set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

elmrt_status hip_fail(hipError_t e, const char* what)
{
    return fail(ELMRT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr int kReadBlocks = elmrt::kReadoutBlocks;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

template <typename T>
void widen(const void* src, double* dst, size_t n)
{
    const T* p = (const T*)src;
    for (size_t i = 0; i < n; ++i) dst[i] = (double)p[i];
}

// ------------------------------------------------------------ thermodynamics

// Peng-Robinson (Sec. 3.1): P = rho R T/(1 - b rho) - a alpha rho^2/(1 + 2 b rho - b^2 rho^2)
struct PengRobinson {
    double RT, b, aal;

    PengRobinson(double a, double b_, double R, double acentric, double Tr)
    {
        const double Tc = 0.0778 * a / (0.45724 * b_ * R);
        const double m = 0.37464 + 1.54226 * acentric - 0.26992 * acentric * acentric;
        const double s = 1.0 + m * (1.0 - std::sqrt(Tr));
        RT = R * Tr * Tc;
        b = b_;
        aal = a * s * s;
    }
    double P(double r) const
    {
        return r * RT / (1.0 - b * r) - aal * r * r / (1.0 + 2.0 * b * r - b * b * r * r);
    }
    double dP(double r) const
    {
        const double g = 1.0 + 2.0 * b * r - b * b * r * r;
        const double dg = 2.0 * b - 2.0 * b * b * r;
        const double om = 1.0 - b * r;
        return RT / (om * om) - aal * (2.0 * r * g - r * r * dg) / (g * g);
    }
    // exact antiderivative of P / rho^2
    double G(double r) const
    {
        const double s2 = std::sqrt(2.0);
        return RT * std::log(r / (1.0 - b * r)) -
               aal / (2.0 * s2 * b) * std::log((1.0 + (1.0 + s2) * b * r) / (1.0 + (1.0 - s2) * b * r));
    }
    // root of P(r) = p on [lo, hi] where P is increasing: safeguarded Newton
    double solve(double p, double lo, double hi) const
    {
        double r = 0.5 * (lo + hi);
        for (int it = 0; it < 200; ++it) {
            const double f = P(r) - p;
            if (f > 0.0) hi = r; else lo = r;
            const double d = dP(r);
            double nr = r - f / d;
            if (!(nr > lo && nr < hi) || !(d > 0.0)) nr = 0.5 * (lo + hi);
            if (std::fabs(nr - r) <= 1e-16 * r) { r = nr; break; }
            r = nr;
        }
        return r;
    }
};

// Maxwell equal-area rule (Sec. 3.1.1) written with the exact antiderivative:
// P_sat (1/rho_v - 1/rho_l) = G(rho_l) - G(rho_v), P(rho_v) = P(rho_l) = P_sat.
bool maxwell(const PengRobinson& pr, double* rv, double* rl, double* ps)
{
    const double rmax = 1.0 / pr.b;
    double s1 = -1.0, s2 = -1.0;
    const int NS = 20000;
    double prev = pr.dP(rmax * 1e-9), prev_r = rmax * 1e-9;
    for (int k = 1; k < NS && s2 < 0.0; ++k) {
        const double r = rmax * k / NS;
        const double d = pr.dP(r);
        if (s1 < 0.0 && prev > 0.0 && d <= 0.0) {
            double lo = prev_r, hi = r;
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + hi);
                (pr.dP(mid) > 0.0 ? lo : hi) = mid;
            }
            s1 = 0.5 * (lo + hi);
        } else if (s1 > 0.0 && prev < 0.0 && d >= 0.0) {
            double lo = prev_r, hi = r;
            for (int it = 0; it < 100; ++it) {
                const double mid = 0.5 * (lo + hi);
                (pr.dP(mid) < 0.0 ? lo : hi) = mid;
            }
            s2 = 0.5 * (lo + hi);
        }
        prev = d;
        prev_r = r;
    }
    if (s1 < 0.0 || s2 < 0.0) return false;
    double lo = std::max(pr.P(s2), 0.0), hi = pr.P(s1);
    double a = 0.0, c = 0.0, p = 0.0;
    for (int it = 0; it < 200; ++it) {
        p = 0.5 * (lo + hi);
        if (p == lo || p == hi) break;
        a = pr.solve(p, 0.0, s1);
        c = pr.solve(p, s2, rmax * (1.0 - 1e-15));
        const double area = p * (1.0 / a - 1.0 / c) - (pr.G(c) - pr.G(a));
        (area > 0.0 ? hi : lo) = p;
    }
    *ps = p;
    *rv = pr.solve(p, 0.0, s1);
    *rl = pr.solve(p, s2, rmax * (1.0 - 1e-15));
    return true;
}

// -------------------------------------------------------------- validation

elmrt_status validate(const elmrt_params* p)
{
    if (!p) return fail(ELMRT_E_INVALID, "params is NULL");
    if (p->struct_size != sizeof(elmrt_params))
        return fail(ELMRT_E_INVALID, "params.struct_size != sizeof(elmrt_params)");
    if (p->lattice != ELMRT_D2Q9 && p->lattice != ELMRT_D3Q27) return fail(ELMRT_E_INVALID, "unknown lattice");
    if (p->precision != ELMRT_FP32 && p->precision != ELMRT_FP64) return fail(ELMRT_E_INVALID, "unknown precision");
    if (p->collision != ELMRT_ENTROPIC && p->collision != ELMRT_BGK) return fail(ELMRT_E_INVALID, "unknown collision");
    const int D = p->lattice == ELMRT_D2Q9 ? 2 : 3;
    for (int a = 0; a < 3; ++a) {
        if (a < D && p->n[a] < 4) return fail(ELMRT_E_INVALID, "grid extent < 4");
        if (a < D && p->bc[a] != ELMRT_PERIODIC && p->bc[a] != ELMRT_WALL) return fail(ELMRT_E_INVALID, "unknown bc");
        if (p->n[a] > 65535 * 16) return fail(ELMRT_E_INVALID, "grid extent too large");
    }
    if (D == 2 && p->n[2] != 1) return fail(ELMRT_E_INVALID, "D2Q9 needs n[2] == 1");
    const long double cells = (long double)p->n[0] * p->n[1] * p->n[2];
    if (cells >= 2147483648.0L) return fail(ELMRT_E_INVALID, "grid has >= 2^31 cells");
    {
        // a plane block (Q populations of one plane normal to the last axis) is
        // addressed with 32-bit offsets
        const long double plane = D == 3 ? (long double)p->n[0] * p->n[1] : (long double)p->n[0];
        const long double block = plane * (D == 3 ? 27 : 9) * (p->precision == ELMRT_FP64 ? 8 : 4);
        if (block >= 2147483648.0L) return fail(ELMRT_E_INVALID, "plane block (Q x cells per plane x value size) >= 2^31 bytes");
    }
    if (!(p->eos_a > 0) || !(p->eos_b > 0) || !(p->eos_R > 0)) return fail(ELMRT_E_INVALID, "EOS a, b, R must be > 0");
    if (!(p->T_over_Tc > 0 && p->T_over_Tc < 1)) return fail(ELMRT_E_INVALID, "T/Tc must be in (0, 1)");
    if (!(p->kappa_tilde >= 0) || !std::isfinite(p->kappa_tilde)) return fail(ELMRT_E_INVALID, "kappa_tilde must be >= 0");
    if (!(p->nu_liquid > 0) || !(p->nu_vapour > 0)) return fail(ELMRT_E_INVALID, "viscosities must be > 0");
    if (p->nu_liquid != p->nu_vapour && !(p->rho_liquid > p->rho_vapour && p->rho_vapour >= 0))
        return fail(ELMRT_E_INVALID, "rho_liquid must exceed rho_vapour when the viscosities differ");
    if (p->readings & ~(ELMRT_READING_TRACE_IN_S | ELMRT_READING_PHI_FLUID_VELOCITY))
        return fail(ELMRT_E_INVALID, "unknown readings bits");
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(p->body_accel[a])) return fail(ELMRT_E_INVALID, "body_accel must be finite");
        if (a >= D && p->body_accel[a] != 0.0) return fail(ELMRT_E_INVALID, "body_accel along an axis the lattice lacks");
    }
    if (!(p->target_W >= 0) || !std::isfinite(p->target_W)) return fail(ELMRT_E_INVALID, "target_W must be >= 0");
    if (p->target_W > 0 && p->kappa_tilde != 0)
        return fail(ELMRT_E_INVALID, "give kappa_tilde or target_W, not both");
    return ELMRT_OK;
}

// Square-gradient capillarity of an interface of width W: kappa~ = 2 max
// omega W^2 / (rho_l - rho_v)^2, omega(rho) = rho [G(rho) - G(rho_v) + P_sat
// (1/rho - 1/rho_v)] with G the antiderivative of P/rho^2.  omega vanishes at
// both Maxwell densities and peaks where mu(rho) = mu_sat between the
// spinodals: a scan, then golden-section refinement of the bracket.
bool kappa_for_width(const PengRobinson& pr, double W, double* kappa)
{
    double rv, rl, ps;
    if (!maxwell(pr, &rv, &rl, &ps)) return false;
    const double Gv = pr.G(rv);
    auto omega = [&](double r) { return r * (pr.G(r) - Gv + ps * (1.0 / r - 1.0 / rv)); };
    const int NS = 4000;
    int kbest = 1;
    double best = -1.0;
    for (int k = 1; k < NS; ++k) {
        const double om = omega(rv + (rl - rv) * k / NS);
        if (om > best) { best = om; kbest = k; }
    }
    double lo = rv + (rl - rv) * (kbest - 1) / NS, hi = rv + (rl - rv) * (kbest + 1) / NS;
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    for (int it = 0; it < 200 && hi - lo > 1e-15 * rl; ++it) {
        const double a = hi - g * (hi - lo), b = lo + g * (hi - lo);
        (omega(a) > omega(b) ? hi : lo) = omega(a) > omega(b) ? b : a;
    }
    best = std::max(best, omega(0.5 * (lo + hi)));
    *kappa = 2.0 * best * W * W / ((rl - rv) * (rl - rv));
    return true;
}

// kappa~ of the problem: as given, or derived from target_W.
bool problem_kappa(const elmrt_params* p, double* kappa)
{
    if (!(p->target_W > 0)) {
        *kappa = p->kappa_tilde;
        return true;
    }
    PengRobinson pr(p->eos_a, p->eos_b, p->eos_R, p->acentric, p->T_over_Tc);
    return kappa_for_width(pr, p->target_W, kappa);
}

struct Layout {
    size_t fA, fB, rho, q, flag, partials, total;
};

Layout layout_of(const elmrt_params* p)
{
    const int D = p->lattice == ELMRT_D2Q9 ? 2 : 3;
    const int Q = D == 2 ? 9 : 27;
    const size_t N = (size_t)p->n[0] * p->n[1] * p->n[2];
    const size_t es = p->precision == ELMRT_FP64 ? 8 : 4;
    Layout L;
    size_t o = 0;
    L.fA = o;       o = align_up(o + (size_t)Q * N * es);
    L.fB = o;       o = align_up(o + (size_t)Q * N * es);
    L.rho = o;      o = align_up(o + N * es);
    L.q = o;        o = align_up(o + (size_t)D * N * es);
    L.flag = o;     o = align_up(o + 256);
    L.partials = o; o = align_up(o + (size_t)kReadBlocks * 8 * sizeof(double));
    L.total = o;
    return L;
}

}  // namespace

struct elmrt_sim {
    elmrt_params p;
    int D, Q;
    size_t N, es;
    char* ws;
    size_t ws_bytes;
    hipStream_t stream;
    void* buf[2];
    int cur;            // index of the buffer holding the state
    void* rho;
    void* q;
    unsigned* flag;
    double* partials;
    bool initialised;
    int device;         // the device current at elmrt_create
    int tx, ty, tm;
    elmrt::Phys<double> ph;
    elmrt::Launch L;
    // header of this sim's state snapshots (constant, so an asynchronous copy
    // may read it at any time)
    struct StateHeader {
        uint64_t magic;
        int32_t lattice, precision, n[3], pad;
        uint64_t pop_bytes;
    } snap{};
};

namespace {
constexpr uint64_t kStateMagic = 0x31455441544d4c45ull;   // "ELMTATE1", little-endian
constexpr size_t kFlagBlock = 256;                         // instability flag + fall-back count
size_t state_bytes_of(const elmrt_sim* s) { return 2 * kAlign + s->Q * s->N * s->es; }
}  // namespace

extern "C" {

elmrt_status elmrt_workspace_bytes(const elmrt_params* p, size_t* bytes)
{
    elmrt_status st = validate(p);
    if (st != ELMRT_OK) return st;
    if (!bytes) return fail(ELMRT_E_INVALID, "bytes is NULL");
    *bytes = layout_of(p).total;
    return ELMRT_OK;
}

elmrt_status elmrt_create(const elmrt_params* p, void* ws, size_t ws_bytes, void* stream, elmrt_sim** out)
{
    elmrt_status st = validate(p);
    if (st != ELMRT_OK) return st;
    if (!out) return fail(ELMRT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!ws) return fail(ELMRT_E_INVALID, "workspace is NULL");
    if ((uintptr_t)ws % kAlign) return fail(ELMRT_E_INVALID, "workspace is not 256-byte aligned");
    const Layout lay = layout_of(p);
    if (ws_bytes < lay.total) return fail(ELMRT_E_NOMEM, "workspace smaller than elmrt_workspace_bytes()");
    elmrt_sim* s = new (std::nothrow) elmrt_sim();
    if (!s) return fail(ELMRT_E_NOMEM, "host allocation failed");
    s->p = *p;
    s->D = p->lattice == ELMRT_D2Q9 ? 2 : 3;
    s->Q = s->D == 2 ? 9 : 27;
    s->N = (size_t)p->n[0] * p->n[1] * p->n[2];
    s->es = p->precision == ELMRT_FP64 ? 8 : 4;
    s->ws = (char*)ws;
    s->ws_bytes = ws_bytes;
    s->stream = (hipStream_t)stream;
    s->buf[0] = s->ws + lay.fA;
    s->buf[1] = s->ws + lay.fB;
    s->cur = 0;
    s->rho = s->ws + lay.rho;
    s->q = s->ws + lay.q;
    s->flag = (unsigned*)(s->ws + lay.flag);
    s->partials = (double*)(s->ws + lay.partials);
    s->initialised = false;
    if (hipGetDevice(&s->device) != hipSuccess) s->device = -1;
    s->tx = 64;
    s->ty = s->D == 3 ? 4 : 1;
    s->tm = 0;   // automatic marching depth (auto_depth)
    s->snap.magic = kStateMagic;
    s->snap.lattice = p->lattice;
    s->snap.precision = p->precision;
    for (int a = 0; a < 3; ++a) s->snap.n[a] = (int32_t)p->n[a];
    s->snap.pop_bytes = (uint64_t)s->Q * s->N * s->es;
    // physics constants (host FP64; cast to the working precision at launch)
    PengRobinson pr(p->eos_a, p->eos_b, p->eos_R, p->acentric, p->T_over_Tc);
    s->ph.RT = pr.RT;
    s->ph.b = pr.b;
    s->ph.aal = pr.aal;
    if (!problem_kappa(p, &s->ph.kappa)) {
        delete s;
        return fail(ELMRT_E_INVALID, "target_W given at a temperature without a two-phase region");
    }
    if (p->nu_liquid == p->nu_vapour) {
        s->ph.nu_v = p->nu_liquid;
        s->ph.dnu = 0.0;
        s->ph.rho_v = 0.0;
        s->ph.inv_drho = 0.0;
    } else {
        s->ph.nu_v = p->nu_vapour;
        s->ph.dnu = p->nu_liquid - p->nu_vapour;
        s->ph.rho_v = p->rho_vapour;
        s->ph.inv_drho = 1.0 / (p->rho_liquid - p->rho_vapour);
    }
    s->ph.entropic = p->collision == ELMRT_ENTROPIC ? 1 : 0;
    s->ph.trace_in_h = (p->readings & ELMRT_READING_TRACE_IN_S) ? 0 : 1;
    s->ph.phi_fluid = (p->readings & ELMRT_READING_PHI_FLUID_VELOCITY) ? 1 : 0;
    for (int a = 0; a < 3; ++a) s->ph.g[a] = p->body_accel[a];
    s->L.D = s->D;
    s->L.fp64 = p->precision == ELMRT_FP64;
    for (int a = 0; a < 3; ++a) {
        s->L.g.n[a] = (int)p->n[a];
        s->L.g.wall[a] = (a < s->D) ? (p->bc[a] == ELMRT_WALL) : 0;
    }
    s->L.g.N = (int)s->N;
    s->L.g.nxny = (int)(p->n[0] * p->n[1]);
    s->L.stream = s->stream;
    hipError_t e = hipMemsetAsync(s->flag, 0, 256, s->stream);
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipMemsetAsync(flag)");
    }
    *out = s;
    return ELMRT_OK;
}

elmrt_status elmrt_init_fields(elmrt_sim* s, const double* rho0, const double* u0)
{
    if (!s || !rho0 || !u0) return fail(ELMRT_E_INVALID, "NULL argument");
    for (size_t c = 0; c < s->N; ++c)
        if (!(rho0[c] > 0.0) || !std::isfinite(rho0[c]))
            return fail(ELMRT_E_INVALID, "rho0 must be finite and positive");
    for (size_t c = 0; c < (size_t)s->D * s->N; ++c)
        if (!std::isfinite(u0[c])) return fail(ELMRT_E_INVALID, "u0 must be finite");
    // stage rho0 and u0 (FP64) in the buffer that does not hold the state
    double* stage = (double*)s->buf[1 - s->cur];
    hipError_t e = hipMemcpyAsync(stage, rho0, s->N * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(stage + s->N, u0, (size_t)s->D * s->N * sizeof(double), hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(init)");
    e = elmrt::launch_shift_velocity(s->L, stage, stage + s->N, s->ph);
    if (e != hipSuccess) return hip_fail(e, "velocity shift kernel");
    e = elmrt::launch_init(s->L, stage, stage + s->N, s->buf[s->cur]);
    if (e != hipSuccess) return hip_fail(e, "init kernel");
    e = hipMemsetAsync(s->flag, 0, 256, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "init");
    s->initialised = true;
    return ELMRT_OK;
}

// Marching depth of the collision tiles.  A deep march amortises the psi
// recomputation on the 4 halo planes of every tile; a shallow one gives small
// launches enough workgroups.  An explicit depth is used as set.  The
// automatic depth of a launch (one grid, or all members of a batch) is the
// deepest of 16, 8, 4, 2, 1 whose launch still holds min_waves wavefronts,
// about two thirds of what the chip holds at each kernel's occupancy (3 per
// SIMD for D3Q27 FP32, 5 for D2Q9); the thresholds are measured on 64^3..256^3
// and 128^2..1024^2 impacts.  Members never march deeper than their grid.
static int member_depth(const elmrt_sim* s, int cap)
{
    return s->tm > 0 ? s->tm : std::min(cap, s->L.g.n[s->D - 1]);
}
static int auto_depth(elmrt_sim* const* sims, size_t count)
{
    if (count == 0) return 16;
    const long long min_waves = sims[0]->D == 3 ? 2048 : 4096;
    int cap = 16;
    for (; cap > 1; cap /= 2) {
        long long waves = 0;
        for (size_t k = 0; k < count; ++k) {
            const elmrt_sim* s = sims[k];
            const long long per_block = (s->tx * s->ty + 63) / 64;
            waves += elmrt::collide_tiling(s->D, s->L.g, s->tx, s->ty, member_depth(s, cap)).blocks * per_block;
        }
        if (waves >= min_waves) break;
    }
    return cap;
}

// Enqueue nsteps steps.  With ev != NULL (2*nsteps + 1 events) an event is
// recorded before the first kernel and after every kernel, so that kernel k
// of the run lies between ev[k] and ev[k+1].
static elmrt_status step_impl(elmrt_sim* s, int64_t nsteps, hipEvent_t* ev)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    if (nsteps < 0) return fail(ELMRT_E_INVALID, "nsteps < 0");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[0], s->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    const int cap = auto_depth(&s, 1);
    for (int64_t k = 0; k < nsteps; ++k) {
        void* cur = s->buf[s->cur];
        void* nxt = s->buf[1 - s->cur];
        e = elmrt::launch_macro(s->L, cur, s->rho, s->q, s->flag, 1.0 / s->ph.b, s->ph.phi_fluid);
        if (e != hipSuccess) return hip_fail(e, "moment kernel");
        if (s->ph.phi_fluid && (e = elmrt::launch_flux_fluid(s->L, s->rho, s->q, s->ph)) != hipSuccess)
            return hip_fail(e, "flux kernel");
        if (ev && (e = hipEventRecord(ev[2 * k + 1], s->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        e = elmrt::launch_collide(s->L, s->tx, s->ty, member_depth(s, cap), cur, nxt, s->rho, s->q, s->ph, s->flag);
        if (e != hipSuccess) return hip_fail(e, "collision kernel");
        if (ev && (e = hipEventRecord(ev[2 * k + 2], s->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        s->cur = 1 - s->cur;
    }
    return ELMRT_OK;
}

elmrt_status elmrt_step(elmrt_sim* s, int64_t nsteps) { return step_impl(s, nsteps, nullptr); }

elmrt_status elmrt_step_timed(elmrt_sim* s, int64_t nsteps, double ms[2])
{
    if (!ms) return fail(ELMRT_E_INVALID, "ms is NULL");
    if (nsteps < 0 || nsteps > (1 << 20)) return fail(ELMRT_E_INVALID, "nsteps out of range for timing");
    ms[0] = ms[1] = 0.0;
    std::vector<hipEvent_t> ev((size_t)(2 * nsteps + 1));
    size_t made = 0;
    hipError_t e = hipSuccess;
    for (; made < ev.size(); ++made)
        if ((e = hipEventCreate(&ev[made])) != hipSuccess) break;
    elmrt_status st = ELMRT_OK;
    if (e != hipSuccess) st = hip_fail(e, "hipEventCreate");
    if (st == ELMRT_OK) st = step_impl(s, nsteps, ev.data());
    if (st == ELMRT_OK && (e = hipEventSynchronize(ev.back())) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
    for (int64_t k = 0; st == ELMRT_OK && k < nsteps; ++k) {
        float a = 0.f, b = 0.f;
        if ((e = hipEventElapsedTime(&a, ev[2 * k], ev[2 * k + 1])) != hipSuccess ||
            (e = hipEventElapsedTime(&b, ev[2 * k + 1], ev[2 * k + 2])) != hipSuccess)
            st = hip_fail(e, "hipEventElapsedTime");
        ms[0] += a;
        ms[1] += b;
    }
    for (size_t k = 0; k < made; ++k) (void)hipEventDestroy(ev[k]);
    return st;
}

static elmrt_status read_impl(elmrt_sim* s, double* rho, double* u, double* sums, bool fluid)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    char* tmp = (char*)s->buf[1 - s->cur];
    void* trho = tmp;
    void* tu = tmp + s->N * s->es;
    hipError_t e = elmrt::launch_readout(s->L, s->buf[s->cur], trho, tu, s->partials, kReadBlocks, s->flag, 1.0 / s->ph.b);
    if (e != hipSuccess) return hip_fail(e, "readout kernel");
    if (fluid && (e = elmrt::launch_fluid_velocity(s->L, trho, tu, s->ph)) != hipSuccess)
        return hip_fail(e, "velocity shift kernel");
    // only the fields asked for cross PCIe (density first, then velocity)
    std::vector<char> h(((u ? 1 + (size_t)s->D : (rho ? 1 : 0))) * s->N * s->es);
    std::vector<double> part((size_t)kReadBlocks * 8);
    unsigned flag = 0;
    e = h.empty() ? hipSuccess : hipMemcpyAsync(h.data(), tmp, h.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(part.data(), s->partials, part.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, s->flag, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "read_macros copy");
    if (rho) {
        if (s->es == 4) widen<float>(h.data(), rho, s->N);
        else widen<double>(h.data(), rho, s->N);
    }
    if (u) {
        if (s->es == 4) widen<float>(h.data() + s->N * s->es, u, (size_t)s->D * s->N);
        else widen<double>(h.data() + s->N * s->es, u, (size_t)s->D * s->N);
    }
    if (sums) {
        // the blocks' (sum, correction) pairs merged in block order by
        // Neumaier's compensated summation, as within the blocks
        for (int k = 0; k < 4; ++k) {
            double acc = 0.0, comp = 0.0;
            for (int b = 0; b < kReadBlocks; ++b) {
                const double x = part[(size_t)b * 8 + 2 * k];
                const double t = acc + x;
                comp += (std::fabs(acc) >= std::fabs(x)) ? (acc - t) + x : (x - t) + acc;
                acc = t;
                comp += part[(size_t)b * 8 + 2 * k + 1];
            }
            sums[k] = acc + comp;
        }
    }
    if (flag) return fail(ELMRT_E_UNSTABLE, "non-finite, non-positive or >= 1/b density encountered");
    return ELMRT_OK;
}

elmrt_status elmrt_read_macros(elmrt_sim* s, double* rho, double* u, double* sums)
{
    return read_impl(s, rho, u, sums, false);
}

elmrt_status elmrt_read_fluid_velocity(elmrt_sim* s, double* u)
{
    if (!u) return fail(ELMRT_E_INVALID, "u is NULL");
    return read_impl(s, nullptr, u, nullptr, true);
}

elmrt_status elmrt_read_sums_noalloc(elmrt_sim* s, double* dev_sums, uint32_t* dev_flag)
{
    if (!s || !dev_sums) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != s->device) return fail(ELMRT_E_INVALID, "the simulation's device must be current");
    double* scratch = nullptr;
    int capacity = 0;
    if ((e = elmrt::readout_scratch(&scratch, &capacity)) != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (kReadBlocks > capacity) return fail(ELMRT_E_INVALID, "read-out reduction larger than the device scratch");
    e = elmrt::launch_readout(s->L, s->buf[s->cur], nullptr, nullptr, scratch, kReadBlocks, s->flag, 1.0 / s->ph.b);
    if (e != hipSuccess) return hip_fail(e, "readout kernel");
    e = elmrt::launch_finish_sums(scratch, kReadBlocks, s->flag, dev_sums, dev_flag, s->stream);
    if (e != hipSuccess) return hip_fail(e, "sums kernel");
    return ELMRT_OK;
}

elmrt_status elmrt_read_populations(elmrt_sim* s, double* f)
{
    if (!s || !f) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    void* tmp = s->buf[1 - s->cur];
    hipError_t e = elmrt::launch_pull(s->L, s->buf[s->cur], tmp);
    if (e != hipSuccess) return hip_fail(e, "pull kernel");
    std::vector<char> h((size_t)s->Q * s->N * s->es);
    e = hipMemcpyAsync(h.data(), tmp, h.size(), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "read_populations copy");
    if (s->es == 4) widen<float>(h.data(), f, (size_t)s->Q * s->N);
    else widen<double>(h.data(), f, (size_t)s->Q * s->N);
    return ELMRT_OK;
}

int32_t elmrt_velocities(int32_t lattice, int32_t* c)
{
    if (lattice != ELMRT_D2Q9 && lattice != ELMRT_D3Q27) return -1;
    const int D = lattice == ELMRT_D2Q9 ? 2 : 3;
    const int Q = D == 2 ? 9 : 27;
    if (c)
        for (int i = 0; i < Q; ++i) {
            c[3 * i + 0] = i % 3 - 1;
            c[3 * i + 1] = (i / 3) % 3 - 1;
            c[3 * i + 2] = D == 3 ? i / 9 - 1 : 0;
        }
    return Q;
}

elmrt_status elmrt_coexistence(const elmrt_params* p, double* rho_vapour, double* rho_liquid, double* p_sat)
{
    if (!p || !rho_vapour || !rho_liquid || !p_sat) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!(p->eos_a > 0) || !(p->eos_b > 0) || !(p->eos_R > 0)) return fail(ELMRT_E_INVALID, "EOS a, b, R must be > 0");
    if (!(p->T_over_Tc > 0 && p->T_over_Tc < 1)) return fail(ELMRT_E_INVALID, "T/Tc must be in (0, 1)");
    PengRobinson pr(p->eos_a, p->eos_b, p->eos_R, p->acentric, p->T_over_Tc);
    if (!maxwell(pr, rho_vapour, rho_liquid, p_sat)) return fail(ELMRT_E_INVALID, "no two-phase region at this temperature");
    return ELMRT_OK;
}

elmrt_status elmrt_kappa_for_width(const elmrt_params* p, double W, double* kappa)
{
    if (!p || !kappa) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!(W > 0) || !std::isfinite(W)) return fail(ELMRT_E_INVALID, "W must be > 0");
    if (!(p->eos_a > 0) || !(p->eos_b > 0) || !(p->eos_R > 0)) return fail(ELMRT_E_INVALID, "EOS a, b, R must be > 0");
    if (!(p->T_over_Tc > 0 && p->T_over_Tc < 1)) return fail(ELMRT_E_INVALID, "T/Tc must be in (0, 1)");
    PengRobinson pr(p->eos_a, p->eos_b, p->eos_R, p->acentric, p->T_over_Tc);
    if (!kappa_for_width(pr, W, kappa)) return fail(ELMRT_E_INVALID, "no two-phase region at this temperature");
    return ELMRT_OK;
}

elmrt_status elmrt_pressure(const elmrt_params* p, const double* rho, double* P, int64_t n)
{
    if (!p || (n > 0 && (!rho || !P))) return fail(ELMRT_E_INVALID, "NULL argument");
    if (n < 0) return fail(ELMRT_E_INVALID, "n < 0");
    if (!(p->eos_a > 0) || !(p->eos_b > 0) || !(p->eos_R > 0)) return fail(ELMRT_E_INVALID, "EOS a, b, R must be > 0");
    if (!(p->T_over_Tc > 0)) return fail(ELMRT_E_INVALID, "T/Tc must be > 0");
    PengRobinson pr(p->eos_a, p->eos_b, p->eos_R, p->acentric, p->T_over_Tc);
    for (int64_t k = 0; k < n; ++k) P[k] = pr.P(rho[k]);
    return ELMRT_OK;
}

elmrt_status elmrt_poll_unstable(elmrt_sim* s, uint32_t* host_word)
{
    if (!s || !host_word) return fail(ELMRT_E_INVALID, "NULL argument");
    const hipError_t e = hipMemcpyAsync(host_word, s->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream);
    if (e != hipSuccess) return hip_fail(e, "poll copy");
    return ELMRT_OK;
}

elmrt_status elmrt_state_bytes(const elmrt_sim* s, size_t* bytes)
{
    if (!s || !bytes) return fail(ELMRT_E_INVALID, "NULL argument");
    *bytes = state_bytes_of(s);
    return ELMRT_OK;
}

// Snapshot layout: [header, 256 B][flag block, 256 B][populations of the
// current state in the library's plane-blocked layout].
elmrt_status elmrt_save_state(elmrt_sim* s, void* dev_dst, size_t bytes)
{
    if (!s || !dev_dst) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    if (bytes < state_bytes_of(s)) return fail(ELMRT_E_INVALID, "snapshot buffer smaller than elmrt_state_bytes()");
    char* d = (char*)dev_dst;
    hipError_t e = hipMemcpyAsync(d, &s->snap, sizeof(s->snap), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d + kAlign, s->flag, kFlagBlock, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d + 2 * kAlign, s->buf[s->cur], s->snap.pop_bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "save_state copy");
    return ELMRT_OK;
}

elmrt_status elmrt_load_state(elmrt_sim* s, const void* dev_src, size_t bytes)
{
    if (!s || !dev_src) return fail(ELMRT_E_INVALID, "NULL argument");
    if (bytes < state_bytes_of(s)) return fail(ELMRT_E_INVALID, "snapshot smaller than elmrt_state_bytes()");
    const char* d = (const char*)dev_src;
    elmrt_sim::StateHeader h{};
    hipError_t e = hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "load_state header");
    if (h.magic != kStateMagic) return fail(ELMRT_E_INVALID, "not a state snapshot");
    if (h.lattice != s->snap.lattice || h.precision != s->snap.precision || h.n[0] != s->snap.n[0] ||
        h.n[1] != s->snap.n[1] || h.n[2] != s->snap.n[2] || h.pop_bytes != s->snap.pop_bytes)
        return fail(ELMRT_E_INVALID, "snapshot of a different lattice, precision or grid");
    e = hipMemcpyAsync(s->flag, d + kAlign, kFlagBlock, hipMemcpyDeviceToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->buf[s->cur], d + 2 * kAlign, s->snap.pop_bytes, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return hip_fail(e, "load_state copy");
    s->initialised = true;
    return ELMRT_OK;
}

elmrt_status elmrt_gamma_fallbacks(elmrt_sim* s, int64_t* cells)
{
    if (!s || !cells) return fail(ELMRT_E_INVALID, "NULL argument");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    unsigned long long n = 0;
    hipError_t e = hipMemcpyAsync(&n, elmrt::gamma_fallbacks(s->flag), sizeof(n), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "gamma fall-back count");
    *cells = (int64_t)n;
    return ELMRT_OK;
}

elmrt_status elmrt_set_stream(elmrt_sim* s, void* stream)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    s->stream = (hipStream_t)stream;
    s->L.stream = s->stream;
    return ELMRT_OK;
}

elmrt_status elmrt_get_tiling(const elmrt_sim* s, int32_t* tx, int32_t* ty, int32_t* tm)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    if (tx) *tx = s->tx;
    if (ty) *ty = s->ty;
    if (tm) *tm = s->tm;
    return ELMRT_OK;
}

elmrt_status elmrt_set_tiling(elmrt_sim* s, int32_t tx, int32_t ty, int32_t tm)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    if (tm < 0) return fail(ELMRT_E_INVALID, "tm must be >= 0 (0: automatic)");
    if (!elmrt::collide_shape_supported(s->D, tx, ty)) return fail(ELMRT_E_INVALID, "tile shape not compiled");
    s->tx = tx;
    s->ty = ty;
    s->tm = tm;
    return ELMRT_OK;
}

}  // extern "C"

// ------------------------------------------------------------- autotuning

namespace {

// Candidate collision tilings of a lattice: every compiled shape with marching
// depths 4 .. 64.
// Compiled tile shapes of a lattice, and marching depths.  The coarse depths
// serve batches (many grids of different sizes) and the first stage of the
// single-grid search; the fine depths (every even depth up to 64) its second
// stage: on one grid the best depth depends on how its tiles fill whole
// rounds of resident workgroups (30 planes on 256^3 D3Q27 FP32 are 4% faster
// than 29 or 31, 5% faster than 16).
std::vector<std::array<int, 2>> tile_shapes(int D)
{
    if (D == 2) return {{64, 1}, {128, 1}, {256, 1}};
    return {{64, 4}, {32, 8}, {64, 2}, {128, 2}};
}
const std::vector<int>& coarse_depths()
{
    static const std::vector<int> d = {1, 2, 4, 8, 16, 32, 64};
    return d;
}
std::vector<int> fine_depths()
{
    std::vector<int> d = {1, 2, 4};
    for (int tm = 6; tm <= 64; tm += 2) d.push_back(tm);
    d.push_back(96);
    d.push_back(128);
    return d;
}
std::vector<std::array<int, 3>> tiling_candidates(int D)
{
    std::vector<std::array<int, 3>> c;
    for (const auto& sh : tile_shapes(D))
        for (int tm : coarse_depths()) c.push_back({sh[0], sh[1], tm});
    return c;
}

// Time 'steps' steps of fn on the stream with HIP events (milliseconds).
template <typename F>
elmrt_status time_steps(hipStream_t stream, F&& fn, float* ms)
{
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    elmrt_status st = ELMRT_OK;
    if ((e = hipEventRecord(a, stream)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
    if (st == ELMRT_OK) st = fn();
    if (st == ELMRT_OK && (e = hipEventRecord(b, stream)) != hipSuccess) st = hip_fail(e, "hipEventRecord");
    if (st == ELMRT_OK && (e = hipEventSynchronize(b)) != hipSuccess) st = hip_fail(e, "hipEventSynchronize");
    if (st == ELMRT_OK && (e = hipEventElapsedTime(ms, a, b)) != hipSuccess) st = hip_fail(e, "hipEventElapsedTime");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

}  // namespace

extern "C" {

elmrt_status elmrt_autotune(elmrt_sim* s, int32_t trial_steps, int64_t* steps_taken)
{
    if (!s) return fail(ELMRT_E_INVALID, "sim is NULL");
    if (trial_steps < 1) return fail(ELMRT_E_INVALID, "trial_steps must be >= 1");
    if (!s->initialised) return fail(ELMRT_E_STATE, "elmrt_init_fields has not been called");
    int64_t taken = 0;
    std::vector<std::pair<float, std::array<int, 3>>> timed;
    auto trial = [&](const std::array<int, 3>& c, int steps, float* ms) -> elmrt_status {
        s->tx = c[0];
        s->ty = c[1];
        s->tm = c[2];
        elmrt_status st = step_impl(s, 1, nullptr);   // first launch of a shape: not timed
        if (st == ELMRT_OK) st = time_steps(s->stream, [&] { return step_impl(s, steps, nullptr); }, ms);
        if (st == ELMRT_OK) taken += 1 + steps;
        return st;
    };
    auto best_of = [&]() {
        return std::min_element(timed.begin(), timed.end(),
                                [](const auto& x, const auto& y) { return x.first < y.first; })->second;
    };
    // stage 1: every shape at the coarse depths; stage 2: the best shape at
    // the fine depths; stage 3: the three fastest again, three times longer
    elmrt_status st = ELMRT_OK;
    float ms = 0.f;
    for (const auto& c : tiling_candidates(s->D)) {
        if ((st = trial(c, trial_steps, &ms)) != ELMRT_OK) return st;
        timed.push_back({ms, c});
    }
    const std::array<int, 3> shape = best_of();
    for (int tm : fine_depths()) {
        if (std::find(coarse_depths().begin(), coarse_depths().end(), tm) != coarse_depths().end()) continue;
        const std::array<int, 3> c{shape[0], shape[1], tm};
        if ((st = trial(c, trial_steps, &ms)) != ELMRT_OK) return st;
        timed.push_back({ms, c});
    }
    std::sort(timed.begin(), timed.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
    timed.resize(std::min<size_t>(3, timed.size()));
    for (auto& t : timed)
        if ((st = trial(t.second, 3 * trial_steps, &t.first)) != ELMRT_OK) return st;
    const std::array<int, 3> arg = best_of();
    s->tx = arg[0];
    s->ty = arg[1];
    s->tm = arg[2];
    if (steps_taken) *steps_taken = taken;
    return ELMRT_OK;
}

// ---------------------------------------------------------------- batches

}  // extern "C"

struct elmrt_batch {
    std::vector<elmrt_sim*> sims;
    int D = 0, fp64 = 0;
    hipStream_t stream = nullptr;
    elmrt::BatchJob* djobs = nullptr;   // device table (caller's workspace)
    std::vector<elmrt::BatchJob> hjobs;
    std::vector<int> order;             // sims[order[k]] is table entry k
    struct Group {
        int tx, ty, first, count;
        long long blocks;
    };
    std::vector<Group> groups;          // collision launches, one per tile shape
    long long mblocks = 0;
    int parity = 0;                     // steps since the table was built, mod 2
    bool use_graph = true;
    bool table_unused = false;          // no kernel has read djobs yet (the request
                                        // loop's fresh tables): upload without
                                        // waiting for the members' stream
    hipGraphExec_t exec = nullptr;      // two steps (parity 0 then 1)
    hipGraph_t graph = nullptr;
    hipStream_t capture = nullptr;      // private stream the graph is captured on
                                        // (the caller's may be the null stream)

    ~elmrt_batch()
    {
        drop_graph();
        if (capture) (void)hipStreamDestroy(capture);
    }
    void drop_graph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

namespace {

size_t batch_table_bytes(int count) { return align_up((size_t)count * sizeof(elmrt::BatchJob)); }

elmrt_status batch_create_impl(elmrt_sim* const* sims, int32_t count, void* ws, size_t ws_bytes,
                               elmrt_batch** out, bool fresh);

// A non-blocking stream of the library's (one per device, created on first
// use) for host-to-device copies that must not wait for compute streams.
hipError_t upload_stream(hipStream_t* out)
{
    static std::mutex mu;
    static hipStream_t streams[elmrt::kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= elmrt::kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && (e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking)) != hipSuccess) return e;
    *out = streams[dev];
    return hipSuccess;
}

// (Re)build the device job table from the sims' current state and tilings.
elmrt_status batch_build(elmrt_batch* b)
{
    const int n = (int)b->sims.size();
    b->order.resize(n);
    for (int k = 0; k < n; ++k) b->order[k] = k;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int i, int j) {
        const elmrt_sim* a = b->sims[i];
        const elmrt_sim* c = b->sims[j];
        return a->tx != c->tx ? a->tx < c->tx : a->ty < c->ty;
    });
    b->hjobs.assign(n, elmrt::BatchJob{});
    b->groups.clear();
    long long mfirst = 0, cfirst = 0;
    const int cap = auto_depth(b->sims.data(), b->sims.size());
    for (int k = 0; k < n; ++k) {
        const elmrt_sim* s = b->sims[b->order[k]];
        if (b->groups.empty() || b->groups.back().tx != s->tx || b->groups.back().ty != s->ty) {
            b->groups.push_back({s->tx, s->ty, k, 0, 0});
            cfirst = 0;
        }
        elmrt::BatchJob& J = b->hjobs[k];
        J.buf[0] = s->buf[0];
        J.buf[1] = s->buf[1];
        J.rho = s->rho;
        J.q = s->q;
        J.flag = s->flag;
        J.g = s->L.g;
        J.ph = s->ph;
        const elmrt::Tiling mt = elmrt::macro_tiling(s->D, s->L.g);
        const int tm = member_depth(s, cap);
        const elmrt::Tiling ct = elmrt::collide_tiling(s->D, s->L.g, s->tx, s->ty, tm);
        J.mbx = mt.bx;
        J.mby = mt.by;
        J.mtm = mt.tm;
        J.cbx = ct.bx;
        J.cby = ct.by;
        J.ctm = tm;
        J.mfirst = (int)mfirst;
        J.cfirst = (int)cfirst;
        J.cblocks = (int)ct.blocks;
        J.cur0 = s->cur;
        mfirst += mt.blocks;
        cfirst += (ct.blocks + 7) / 8 * 8;   // ranges start on multiples of 8 (one per XCD)
        b->groups.back().count += 1;
        b->groups.back().blocks = cfirst;
        if (mfirst > 0x7fffffffLL || cfirst > 0x7fffffffLL) return fail(ELMRT_E_INVALID, "batch has >= 2^31 tiles");
    }
    b->mblocks = mfirst;
    b->parity = 0;
    b->drop_graph();
    // A table that kernels enqueued earlier may still read is replaced only
    // after the members' stream has drained; a table no kernel has read yet
    // goes up on the library's own upload stream, without waiting for the
    // compute already enqueued.
    hipStream_t up = b->stream;
    if (b->table_unused) {
        hipError_t e = upload_stream(&up);
        if (e != hipSuccess) return hip_fail(e, "upload stream");
    }
    hipError_t e = hipMemcpyAsync(b->djobs, b->hjobs.data(), (size_t)n * sizeof(elmrt::BatchJob),
                                  hipMemcpyHostToDevice, up);
    if (e == hipSuccess) e = hipStreamSynchronize(up);
    if (e != hipSuccess) return hip_fail(e, "job table upload");
    b->table_unused = false;
    return ELMRT_OK;
}

// One batched step at the given parity: the moment pass over every job, then
// one collision launch per tile shape.
elmrt_status batch_enqueue_step(elmrt_batch* b, int parity, hipStream_t stream)
{
    hipError_t e = elmrt::launch_macro_batch(b->D, b->fp64, b->djobs, (int)b->hjobs.size(), b->mblocks, parity,
                                             stream);
    if (e != hipSuccess) return hip_fail(e, "batched moment kernel");
    // members whose Phi flux takes the fluid velocity: their flux pass, one
    // launch each, once every density of the member is known
    for (const elmrt_sim* s : b->sims) {
        if (!s->ph.phi_fluid) continue;
        elmrt::Launch L = s->L;
        L.stream = stream;
        if ((e = elmrt::launch_flux_fluid(L, s->rho, s->q, s->ph)) != hipSuccess) return hip_fail(e, "flux kernel");
    }
    for (const auto& G : b->groups) {
        e = elmrt::launch_collide_batch(b->D, b->fp64, G.tx, G.ty, b->djobs + G.first, G.count, G.blocks, parity,
                                        stream);
        if (e != hipSuccess) return hip_fail(e, "batched collision kernel");
    }
    return ELMRT_OK;
}

// The sims' buffer indices still match the table (nobody stepped them alone).
bool batch_in_sync(const elmrt_batch* b)
{
    for (size_t k = 0; k < b->hjobs.size(); ++k)
        if (b->sims[b->order[k]]->cur != (b->hjobs[k].cur0 ^ b->parity)) return false;
    return true;
}

elmrt_status batch_capture(elmrt_batch* b)
{
    hipError_t e;
    if (!b->capture && (e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    elmrt_status st = batch_enqueue_step(b, 0, b->capture);
    if (st == ELMRT_OK) st = batch_enqueue_step(b, 1, b->capture);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->capture, &g);
    if (st != ELMRT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->drop_graph();
        return hip_fail(e, "hipGraphInstantiate");
    }
    return ELMRT_OK;
}

elmrt_status batch_step_impl(elmrt_batch* b, int64_t nsteps)
{
    if (!batch_in_sync(b)) {
        elmrt_status st = batch_build(b);
        if (st != ELMRT_OK) return st;
    }
    int64_t k = 0;
    auto advance = [&](int64_t n) {
        b->parity ^= (int)(n & 1);
        for (elmrt_sim* s : b->sims) s->cur ^= (int)(n & 1);
    };
    if (k < nsteps && b->parity == 1) {   // graph replays start at parity 0
        elmrt_status st = batch_enqueue_step(b, 1, b->stream);
        if (st != ELMRT_OK) return st;
        advance(1);
        ++k;
    }
    if (b->use_graph && nsteps - k >= 2) {
        if (!b->exec) {
            elmrt_status st = batch_capture(b);
            if (st != ELMRT_OK) return st;
        }
        for (; nsteps - k >= 2; k += 2) {
            hipError_t e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
            advance(2);
        }
    }
    for (; k < nsteps; ++k) {
        elmrt_status st = batch_enqueue_step(b, b->parity, b->stream);
        if (st != ELMRT_OK) return st;
        advance(1);
    }
    return ELMRT_OK;
}

}  // namespace

extern "C" {

elmrt_status elmrt_batch_workspace_bytes(int32_t count, size_t* bytes)
{
    if (count < 1) return fail(ELMRT_E_INVALID, "count must be >= 1");
    if (!bytes) return fail(ELMRT_E_INVALID, "bytes is NULL");
    *bytes = batch_table_bytes(count);
    return ELMRT_OK;
}

}  // extern "C"

// The request loop's batches: a workspace no kernel has touched yet (the loop
// releases a table's memory only after the rounds that read it have
// completed), so the table goes up without waiting for the compute stream;
// and no graph, since such a batch lives for a few rounds.
elmrt_status elmrt::batch_create_fresh(elmrt_sim* const* sims, int32_t count, void* ws, size_t ws_bytes,
                                       elmrt_batch** out)
{
    return batch_create_impl(sims, count, ws, ws_bytes, out, true);
}

extern "C" {

elmrt_status elmrt_batch_create(elmrt_sim* const* sims, int32_t count, void* ws, size_t ws_bytes,
                                elmrt_batch** out)
{
    return batch_create_impl(sims, count, ws, ws_bytes, out, false);
}

}  // extern "C"

namespace {
elmrt_status batch_create_impl(elmrt_sim* const* sims, int32_t count, void* ws, size_t ws_bytes,
                               elmrt_batch** out, bool fresh)
{
    if (!out) return fail(ELMRT_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!sims || count < 1) return fail(ELMRT_E_INVALID, "no sims");
    if (!ws || ((uintptr_t)ws % kAlign) != 0) return fail(ELMRT_E_INVALID, "workspace is NULL or not 256-byte aligned");
    if (ws_bytes < batch_table_bytes(count)) return fail(ELMRT_E_INVALID, "workspace too small for the job table");
    std::vector<elmrt_sim*> v(sims, sims + count);
    for (int k = 0; k < count; ++k) {
        const elmrt_sim* s = v[k];
        if (!s) return fail(ELMRT_E_INVALID, "a sim is NULL");
        if (!s->initialised) return fail(ELMRT_E_STATE, "a sim has not been initialised");
        if (s->D != v[0]->D || s->L.fp64 != v[0]->L.fp64)
            return fail(ELMRT_E_INVALID, "sims of a batch must share lattice and precision");
        if (s->stream != v[0]->stream) return fail(ELMRT_E_INVALID, "sims of a batch must share the stream");
        for (int j = 0; j < k; ++j)
            if (v[j] == s) return fail(ELMRT_E_INVALID, "a sim appears twice in the batch");
    }
    elmrt_batch* b = new elmrt_batch;
    b->sims = v;
    b->D = v[0]->D;
    b->fp64 = v[0]->L.fp64;
    b->stream = v[0]->stream;
    b->djobs = (elmrt::BatchJob*)ws;
    b->table_unused = fresh;
    b->use_graph = !fresh;
    elmrt_status st = batch_build(b);
    if (st != ELMRT_OK) {
        delete b;
        return st;
    }
    *out = b;
    return ELMRT_OK;
}
}  // namespace

extern "C" {

elmrt_status elmrt_batch_step(elmrt_batch* b, int64_t nsteps)
{
    if (!b) return fail(ELMRT_E_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(ELMRT_E_INVALID, "nsteps < 0");
    for (const elmrt_sim* s : b->sims)
        if (s->stream != b->stream) return fail(ELMRT_E_STATE, "a member was moved to another stream");
    return batch_step_impl(b, nsteps);
}

elmrt_status elmrt_batch_set_graph(elmrt_batch* b, int32_t use_graph)
{
    if (!b) return fail(ELMRT_E_INVALID, "batch is NULL");
    b->use_graph = use_graph != 0;
    return ELMRT_OK;
}

elmrt_status elmrt_batch_autotune(elmrt_batch* b, int32_t trial_steps, int64_t* steps_taken)
{
    if (!b) return fail(ELMRT_E_INVALID, "batch is NULL");
    if (trial_steps < 2) return fail(ELMRT_E_INVALID, "trial_steps must be >= 2");
    int64_t taken = 0;
    float best = 0.f;
    std::vector<std::array<int, 3>> keep;
    for (elmrt_sim* s : b->sims) keep.push_back({s->tx, s->ty, s->tm});
    std::vector<std::array<int, 3>> arg = keep;
    for (const auto& c : tiling_candidates(b->D)) {
        for (elmrt_sim* s : b->sims) {
            s->tx = c[0];
            s->ty = c[1];
            // no deeper than the grid: marching depth at most the last extent
            s->tm = std::min(c[2], s->L.g.n[s->D - 1]);
        }
        elmrt_status st = batch_build(b);
        if (st == ELMRT_OK) st = batch_step_impl(b, 2);   // first replay of a shape: not timed
        float ms = 0.f;
        if (st == ELMRT_OK) st = time_steps(b->stream, [&] { return batch_step_impl(b, trial_steps); }, &ms);
        if (st != ELMRT_OK) return st;
        taken += 2 + trial_steps;
        if (best == 0.f || ms < best) {
            best = ms;
            arg.clear();
            for (elmrt_sim* s : b->sims) arg.push_back({s->tx, s->ty, s->tm});
        }
    }
    for (size_t k = 0; k < b->sims.size(); ++k) {
        b->sims[k]->tx = arg[k][0];
        b->sims[k]->ty = arg[k][1];
        b->sims[k]->tm = arg[k][2];
    }
    elmrt_status st = batch_build(b);
    if (st != ELMRT_OK) return st;
    if (steps_taken) *steps_taken = taken;
    return ELMRT_OK;
}

void elmrt_batch_destroy(elmrt_batch* b) { delete b; }

void elmrt_destroy(elmrt_sim* s) { delete s; }

const char* elmrt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
