// elmrt_kernels.hip -- gfx950 kernels of one time step of the entropic
// multi-relaxation-time two-phase lattice Boltzmann model (Hosseini, Dorschner
// & Karlin, arXiv:2201.12404).
//
// State layout (device, structure of arrays): cur[i*N + cell], cell = x +
// nx*(y + ny*z).  The buffer holds post-collision populations f'(r, t-1) at the
// cell they leave from, so the populations of time t are gathered by pulling:
//   f_i(r, t) = cur_i(r - c_i)        (periodic wrap), or
//   f_i(r, t) = cur_{-i}(r)           (half-way bounce-back when r - c_i is
//                                      behind a wall).
//
// One step = two kernels.
//   k_macro   : pull, rho = sum f, rho u = sum c f (Sec. 2.2), and the flux
//               q_a = rho u_a (u_a^2 + 3 P0/rho - 3 cs^2) = rho u_a^3 with
//               P0 = rho cs^2, whose derivative gives Phi (Sec. 2.2).
//   k_collide : workgroup tile of TX x TY cells marching along the last axis;
//               density planes with a 2-cell halo are staged in LDS together
//               with the signed pseudo-potential psi (Sec. 2.3), computed once
//               per staged cell from the Peng-Robinson pressure (Sec. 3.1).
//               Per cell: the psi and capillary stencils (Sec. 2.3), Phi, the
//               relaxation rate, f^eq and f* in product form (Sec. 2.1-2.2),
//               the s/h split in the modified central Hermite basis
//               (Appendix A) through one-dimensional dual functions, gamma
//               from the entropic scalar products weighted by 1/f* (Sec. 2.4),
//               and f' = f* + (1-omega) s + (1 - omega gamma/2) h, which is the
//               LBGK update with the entropic mirror state written out.
//
// No MFMA: the step is bound by memory traffic, not by contractions.
#include "elmrt_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace elmrt {
namespace {

template <int D>
struct Lat {
    static constexpr int Q = (D == 2) ? 9 : 27;
};

template <int D>
__host__ __device__ constexpr int cx_(int i) { return i % 3 - 1; }
template <int D>
__host__ __device__ constexpr int cy_(int i) { return (i / 3) % 3 - 1; }
template <int D>
__host__ __device__ constexpr int cz_(int i) { return D == 3 ? i / 9 - 1 : 0; }

// Unsigned 32-bit division by a run-time constant (Granlund-Montgomery).
struct FastDiv {
    uint32_t d, m, l;
};

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    return f;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    uint32_t t = __umulhi(n, f.m);
    return (t + n) >> f.l;
}

// Coordinate mapping onto the grid along one axis: periodic wrap, or mirror
// about the wall planes at -1/2 and n-1/2 (period 2n; an odd number of
// reflections toggles *flip).  Every result lies in [0, n).
__device__ __forceinline__ int map_coord(int x, int n, int wall, int* flip)
{
    if (!wall) {
        x %= n;
        return x < 0 ? x + n : x;
    }
    const int p = 2 * n;
    int r = x % p;
    r = r < 0 ? r + p : r;
    if (r >= n) {
        *flip ^= 1;
        return p - 1 - r;
    }
    return r;
}

// Pull addressing of one cell: source offsets and validity per axis and
// per velocity component c (index c + 1).
struct PullIdx {
    int off[3][3];
    bool ok[3][3];
    int self;
};

template <int D>
__device__ __forceinline__ void pull_setup(const Grid& g, int x, int y, int z, PullIdx& P)
{
    const int co[3] = {x, y, z};
    const int st[3] = {1, g.n[0], g.nxny};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (a >= D) {
                P.off[a][k] = 0;
                P.ok[a][k] = true;
                continue;
            }
            const int n = g.n[a];
            int s = co[a] - (k - 1);
            bool ok = true;
            if (!g.wall[a]) {
                s = s < 0 ? s + n : (s >= n ? s - n : s);
            } else {
                ok = (s >= 0) && (s < n);
                s = ok ? s : co[a];
            }
            P.off[a][k] = s * st[a];
            P.ok[a][k] = ok;
        }
    }
    P.self = x + g.n[0] * y + g.nxny * z;
}

template <int D, typename T>
__device__ __forceinline__ void pull(const T* __restrict__ cur, const Grid& g, const PullIdx& P,
                                     T (&f)[Lat<D>::Q])
{
    constexpr int Q = Lat<D>::Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int a = cx_<D>(i) + 1, b = cy_<D>(i) + 1, c = cz_<D>(i) + 1;
        const bool ok = P.ok[0][a] && P.ok[1][b] && P.ok[2][c];
        const int src = P.off[0][a] + P.off[1][b] + P.off[2][c];
        // bounce-back: the population that left r towards the wall, reversed
        const size_t idx = ok ? (size_t)i * g.N + src : (size_t)(Q - 1 - i) * g.N + P.self;
        f[i] = cur[idx];
    }
}

// rho = sum f, j = sum c f, accumulated in A in a fixed order (identical
// wherever it is used).
template <int D, typename T, typename A>
__device__ __forceinline__ void moments(const T (&f)[Lat<D>::Q], A& rho, A (&j)[3])
{
    constexpr int Q = Lat<D>::Q;
    A r = A(0), jx = A(0), jy = A(0), jz = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) r += (A)f[i];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cx_<D>(i) > 0) jx += (A)f[i];
        if (cx_<D>(i) < 0) jx -= (A)f[i];
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cy_<D>(i) > 0) jy += (A)f[i];
        if (cy_<D>(i) < 0) jy -= (A)f[i];
    }
    if (D == 3) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (cz_<D>(i) > 0) jz += (A)f[i];
            if (cz_<D>(i) < 0) jz -= (A)f[i];
        }
    }
    rho = r;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
}

template <typename T>
struct V2 {
    T rho;
    T psi;   // signed pseudo-potential: +psi where P <= P0, -psi where P > P0
};

// Reciprocal and square root: the hardware instructions in FP32 (1 ulp),
// correctly rounded in FP64.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename T>
__device__ __forceinline__ T root(T x);
template <>
__device__ __forceinline__ float root<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double root<double>(double x) { return sqrt(x); }

// psi = sqrt(|P - P0|) (Sec. 2.3), P from the Peng-Robinson EOS (Sec. 3.1),
// P0 = rho cs^2; the sign is the sign of the psi term of the force.
template <typename T>
__device__ __forceinline__ T psi_signed(T r, const Phys<T>& ph)
{
    const T P = r * ph.RT * rcp<T>(T(1) - ph.b * r) -
                ph.aal * r * r * rcp<T>(T(1) + T(2) * ph.b * r - ph.b * ph.b * r * r);
    const T d = P - r * (T(1) / T(3));
    const T s = root<T>(fabs(d));
    return d > T(0) ? -s : s;
}

template <typename T>
__device__ __forceinline__ T omega_of(T r, const Phys<T>& ph)
{
    T x = (r - ph.rho_v) * ph.inv_drho;
    x = x < T(0) ? T(0) : (x > T(1) ? T(1) : x);
    const T nu = ph.nu_v + ph.dnu * x;
    return rcp<T>(T(3) * nu + T(0.5));
}

template <typename T>
__device__ __forceinline__ T pick(const T (&v)[3], int c)
{
    return c == 0 ? v[1] : (c > 0 ? v[2] : v[0]);
}

template <typename T>
struct Eps2;
template <>
struct Eps2<float> {
    static constexpr float v = 3.5527136788005009e-15f;   // (2^-24)^2
};
template <>
struct Eps2<double> {
    static constexpr double v = 1.2325951644078310e-32;   // (2^-53)^2
};

// Storage rounding of the post-collision populations breaks the exact mass
// conservation of the collision (sum f' = rho) by a few ulps per cell and
// step, with a sign that repeats in slowly varying regions, so the mass
// drifts.  The residual is formed in FP64 and absorbed by the rest population.
template <int D, typename T, typename A>
__device__ __forceinline__ void conserve_mass(T (&f)[Lat<D>::Q], A rho)
{
    constexpr int Q = Lat<D>::Q;
    constexpr int REST = (Q - 1) / 2;
    A M = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (i != REST) M += (A)f[i];
    f[REST] = (T)(rho - M);
}

// Collision of one cell.  f: pulled populations (overwritten with f').
// Storage is T.  The per-cell scalars (moments, velocity, force terms, Phi,
// omega, the per-axis factors of the product forms) and the large
// per-population terms f^eq and f* are formed in A (FP64); the small terms
// f - f^eq, s, h and the scalar products stay in T; f' is rounded once.  In
// FP32 this keeps the macroscopic fields within ~1e-6 of the FP64 result over
// 1000 steps, where all-FP32 arithmetic drifts by ~5e-5 (low-density
// interface cells, where the bare velocity and F/rho are O(1) and nearly
// cancel, are the most sensitive).
template <int D, typename T, typename A>
__device__ __forceinline__ void collide(T (&f)[Lat<D>::Q], A rho, const A (&j)[3], const A (&F)[3],
                                        const A (&Phi)[3], A omega, int entropic)
{
    constexpr int Q = Lat<D>::Q;
    const A third = A(1) / A(3);
    const A inv_rho = rcp<A>(rho);
    A u[3] = {A(0), A(0), A(0)};
    A e[3][3], gs[3][3];
    T ef[3][3];
    bool pos = rho > A(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= D) {
            e[a][0] = e[a][2] = gs[a][0] = gs[a][2] = A(0);
            e[a][1] = gs[a][1] = A(1);
            ef[a][0] = ef[a][2] = T(0); ef[a][1] = T(1);
            continue;
        }
        u[a] = j[a] * inv_rho;
        const A zeta = third + u[a] * u[a];
        e[a][1] = A(1) - zeta;
        e[a][2] = A(0.5) * (zeta + u[a]);
        e[a][0] = A(0.5) * (zeta - u[a]);
        const A xs = u[a] + F[a] * inv_rho;
        const A zs = third + xs * xs + Phi[a] * inv_rho;
        gs[a][1] = A(1) - zs;
        gs[a][2] = A(0.5) * (zs + xs);
        gs[a][0] = A(0.5) * (zs - xs);
        pos = pos && gs[a][0] > A(0) && gs[a][1] > A(0) && gs[a][2] > A(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) ef[a][k] = (T)e[a][k];
    }
    // pass 1: f - f^eq (f^eq formed in A; the difference is small) and its second moments
    T Pxx = T(0), Pyy = T(0), Pzz = T(0), Pxy = T(0), Pxz = T(0), Pyz = T(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
        const A feq = rho * e[0][cx + 1] * e[1][cy + 1] * e[2][cz + 1];
        const T fn = (T)((A)f[i] - feq);
        f[i] = fn;
        if (cx) Pxx += fn;
        if (cy) Pyy += fn;
        if (cz) Pzz += fn;
        if (cx * cy > 0) Pxy += fn;
        if (cx * cy < 0) Pxy -= fn;
        if (cx * cz > 0) Pxz += fn;
        if (cx * cz < 0) Pxz -= fn;
        if (cy * cz > 0) Pyz += fn;
        if (cy * cz < 0) Pyz -= fn;
    }
    const T om1 = (T)(A(1) - omega);
    T ch = T(0);
    if (entropic) {
        const T tr = (D == 3) ? (Pxx + Pyy + Pzz) * (T(1) / T(3)) : (Pxx + Pyy) * T(0.5);
        Pxx -= tr;
        Pyy -= tr;
        Pzz = (D == 3) ? Pzz - tr : T(0);
    }
    T p1[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p1[a][0] = (T)(u[a] - A(0.5));
        p1[a][1] = (T)(A(-2) * u[a]);
        p1[a][2] = (T)(u[a] + A(0.5));
    }
    const T p2[3] = {T(0.5), T(-1), T(0.5)};
    auto s_of = [&](int cx, int cy, int cz) -> T {
        const T ex = ef[0][cx + 1], ey = ef[1][cy + 1], ez = ef[2][cz + 1];
        const T px = p1[0][cx + 1], py = p1[1][cy + 1], pz = p1[2][cz + 1];
        T s = Pxx * p2[cx + 1] * ey * ez + Pyy * ex * p2[cy + 1] * ez + Pxy * px * py * ez;
        if (D == 3) s += Pzz * ex * ey * p2[cz + 1] + Pxz * px * ey * pz + Pyz * ex * py * pz;
        return s;
    };
    if (entropic) {
        T ig[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < 3; ++k) ig[a][k] = (a >= D) ? T(1) : (T)rcp<A>(gs[a][k]);
        const T irt = (T)inv_rho;
        T S = T(0), H = T(0);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
            const T s = s_of(cx, cy, cz);
            const T h = f[i] - s;
            const T w = irt * ig[0][cx + 1] * ig[1][cy + 1] * ig[2][cz + 1];
            const T hw = h * w;
            S += s * hw;
            H += h * hw;
        }
        ch = (pos && (A)H > Eps2<A>::v * rho) ? (T)(omega - A(1)) * S * rcp<T>(H) : T(0);
    }
    // f' = f* + (1 - omega) s + (1 - omega gamma/2) h, h = (f - f^eq) - s; BGK: s = 0, h = f - f^eq
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
        const T s = entropic ? s_of(cx, cy, cz) : T(0);
        const A fs = rho * gs[0][cx + 1] * gs[1][cy + 1] * gs[2][cz + 1];
        const T small = entropic ? (om1 * s + ch * (f[i] - s)) : om1 * f[i];
        f[i] = (T)(fs + (A)small);
    }
    if constexpr (sizeof(T) < sizeof(A)) conserve_mass<D, T, A>(f, rho);
}

// ------------------------------------------------------------------ kernels

struct FlatGrid {
    FastDiv nx, ny;
};

__device__ __forceinline__ void flat_coords(uint32_t cell, const FlatGrid& fg, int& x, int& y, int& z)
{
    const uint32_t row = fdiv(cell, fg.nx);
    x = (int)(cell - row * fg.nx.d);
    const uint32_t zz = fdiv(row, fg.ny);
    y = (int)(row - zz * fg.ny.d);
    z = (int)zz;
}

// ----------------------------------------------------- marching tiles
//
// Both step kernels walk a TX x TY tile of the plane normal to the last axis
// (x-y in 3-D, x in 2-D) through tm consecutive planes of that axis.  The
// coordinate along the marching axis is the same for the whole workgroup, so
// its offsets and wall tests are scalar; the in-plane offsets are computed
// once per thread and reused for every plane.

// Raw buffer resource over one plane [base, base + bytes): loads and stores
// take a 32-bit per-lane byte offset and a scalar resource, so no 64-bit
// address is formed per lane; an offset outside the plane reads 0 and writes
// nothing instead of touching other memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
template <>
__device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t off, T v);
template <>
__device__ __forceinline__ void bst<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}
template <>
__device__ __forceinline__ void bst<double>(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    using u2 = __attribute__((ext_vector_type(2))) uint32_t;
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)off, 0, 0);
}

// In-plane pull sources of one lane, source coordinate x - c (c = -1, 0, +1),
// as byte offsets within a plane.
struct LanePull {
    uint32_t xo[3], yo[3];  // yo = 0 in 2-D
    bool xok[3], yok[3];    // false where the source lies behind a wall
    uint32_t ip;            // the cell itself
};

// Marching-axis sources (uniform over the workgroup), as element offsets.
struct PlanePull {
    int mo[3];
    bool mok[3];
    int mself;
    uint32_t bytes;       // bytes of one plane
};

__device__ __forceinline__ void axis_sources(int co, int n, int wall, int stride, int (&o)[3], bool (&ok)[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        int s = co - (k - 1);
        bool v = true;
        if (!wall) {
            s = s < 0 ? s + n : (s >= n ? s - n : s);
        } else {
            v = (s >= 0) && (s < n);
            s = v ? s : co;
        }
        o[k] = s * stride;
        ok[k] = v;
    }
}

template <int D, typename T>
__device__ __forceinline__ void lane_setup(const Grid& g, int x, int y, LanePull& L)
{
    int xo[3], yo[3] = {0, 0, 0};
    axis_sources(x, g.n[0], g.wall[0], 1, xo, L.xok);
    if (D == 3) {
        axis_sources(y, g.n[1], g.wall[1], g.n[0], yo, L.yok);
    } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) L.yok[k] = true;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        L.xo[k] = (uint32_t)xo[k] * (uint32_t)sizeof(T);
        L.yo[k] = (uint32_t)yo[k] * (uint32_t)sizeof(T);
    }
    L.ip = L.xo[1] + L.yo[1];
}

template <int D, typename T>
__device__ __forceinline__ void plane_setup(const Grid& g, int m, PlanePull& P)
{
    const int MA = D - 1;
    const int stride = (D == 3) ? g.nxny : g.n[0];
    axis_sources(m, g.n[MA], g.wall[MA], stride, P.mo, P.mok);
    P.mself = m * stride;
    P.bytes = (uint32_t)stride * (uint32_t)sizeof(T);
}

// Gather f_i(r, t) of one cell.  FAST: no source of this workgroup and plane
// lies behind a wall (no bounce-back selects needed).
template <int D, typename T, bool FAST>
__device__ __forceinline__ void pull_m(const T* __restrict__ cur, int N, const LanePull& L, const PlanePull& P,
                                       T (&f)[Lat<D>::Q])
{
    constexpr int Q = Lat<D>::Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i) + 1, cy = cy_<D>(i) + 1, cz = cz_<D>(i) + 1;
        const int cm = (D == 3) ? cz : cy;           // component along the marching axis
        const uint32_t off = L.xo[cx] + ((D == 3) ? L.yo[cy] : 0u);
        const auto r = plane_rsrc(cur + (size_t)i * N + P.mo[cm], P.bytes);
        if (FAST) {
            f[i] = bld<T>(r, off);
        } else {
            const bool ok = L.xok[cx] && ((D == 3) ? L.yok[cy] : true) && P.mok[cm];
            // bounce-back: the population that left r towards the wall, reversed
            const auto rb = plane_rsrc(cur + (size_t)(Q - 1 - i) * N + P.mself, P.bytes);
            f[i] = ok ? bld<T>(r, off) : bld<T>(rb, L.ip);
        }
    }
}

// Workgroup-uniform test: every active lane of the tile has all in-plane
// sources inside the grid.
template <int D, int TX, int TY>
__device__ __forceinline__ bool tile_clear(const Grid& g, int x0, int y0)
{
    bool c = !g.wall[0] || (x0 >= 1 && x0 + TX <= g.n[0] - 1);
    if (D == 3) c = c && (!g.wall[1] || (y0 >= 1 && y0 + TY <= g.n[1] - 1));
    return c;
}

struct TileCoords {
    int x0, y0, m0, m1;
};

template <int D, int TX, int TY>
__device__ __forceinline__ TileCoords tile_of(const Grid& g, int bx, int by, int tm)
{
    int b = blockIdx.x;
    TileCoords t;
    const int xb = b % bx;
    b /= bx;
    int yb = 0;
    if (D == 3) {
        yb = b % by;
        b /= by;
    }
    t.x0 = xb * TX;
    t.y0 = yb * TY;
    t.m0 = b * tm;
    t.m1 = min(t.m0 + tm, g.n[D - 1]);
    return t;
}

// Moment pass: rho and the Phi flux q_a = rho u_a^3 of every cell.
template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_macro(const T* __restrict__ cur, T* __restrict__ rho_out,
                                                  T* __restrict__ q_out, unsigned* __restrict__ flag,
                                                  Grid g, int bx, int by, int tm)
{
    constexpr int Q = Lat<D>::Q;
    const TileCoords t = tile_of<D, TX, TY>(g, bx, by, tm);
    const int x = t.x0 + (int)threadIdx.x;
    const int y = (D == 3) ? t.y0 + (int)threadIdx.y : 0;
    if (x >= g.n[0] || (D == 3 && y >= g.n[1])) return;
    LanePull L;
    lane_setup<D, T>(g, x, y, L);
    const bool clear = tile_clear<D, TX, TY>(g, t.x0, t.y0);
    bool bad = false;
#pragma unroll 1
    for (int m = t.m0; m < t.m1; ++m) {
        PlanePull P;
        plane_setup<D, T>(g, m, P);
        T f[Q];
        if (clear && P.mok[0] && P.mok[2]) pull_m<D, T, true>(cur, g.N, L, P, f);
        else pull_m<D, T, false>(cur, g.N, L, P, f);
        double rho, j[3];
        moments<D, T, double>(f, rho, j);
        bst<T>(plane_rsrc(rho_out + P.mself, P.bytes), L.ip, (T)rho);
        const double inv = rcp<double>(rho);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double ua = j[a] * inv;
            bst<T>(plane_rsrc(q_out + (size_t)a * g.N + P.mself, P.bytes), L.ip, (T)(j[a] * ua * ua));
        }
        bad = bad || !(rho > 0.0) || !isfinite(rho);
    }
    if (bad) atomicOr(flag, 1u);
}

// Fused stencil + collision pass.
template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_collide(const T* __restrict__ cur, T* __restrict__ nxt,
                                                    const T* __restrict__ rho, const T* __restrict__ q,
                                                    Grid g, Phys<double> ph, int bx, int by, int tm)
{
    constexpr int Q = Lat<D>::Q;
    constexpr int HX = TX + 4;
    constexpr int HY = (D == 3) ? TY + 4 : 1;
    constexpr int NT = TX * TY;
    constexpr int NE = (HX * HY + NT - 1) / NT;   // halo entries staged per thread and plane
    constexpr int MA = D - 1;
    __shared__ V2<T> tile[5][HY][HX];

    const TileCoords t = tile_of<D, TX, TY>(g, bx, by, tm);
    const int tx = threadIdx.x;
    const int ty = (D == 3) ? (int)threadIdx.y : 0;
    const int lid = threadIdx.x + TX * threadIdx.y;
    const int x = t.x0 + tx;
    const int y = (D == 3) ? t.y0 + ty : 0;
    const bool active = (x < g.n[0]) && (D == 2 || y < g.n[1]);
    const int mstride = (D == 3) ? g.nxny : g.n[0];

    // in-plane source (byte offset) of each staged halo entry, fixed for all planes
    int hoff[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int e = lid + k * NT;
        hoff[k] = -1;
        if (e < HX * HY) {
            int dummy = 0;
            const int hx = e % HX, hy = e / HX;
            const int gx = map_coord(t.x0 - 2 + hx, g.n[0], g.wall[0], &dummy);
            const int gy = (D == 3) ? map_coord(t.y0 - 2 + hy, g.n[1], g.wall[1], &dummy) : 0;
            hoff[k] = (gx + g.n[0] * gy) * (int)sizeof(T);
        }
    }
    auto load_plane = [&](int slot, int m) {
        int dummy = 0;
        const auto rp = plane_rsrc(rho + (size_t)map_coord(m, g.n[MA], g.wall[MA], &dummy) * mstride,
                                   (uint32_t)mstride * (uint32_t)sizeof(T));
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            if (hoff[k] >= 0) {
                const int e = lid + k * NT;
                const T r = bld<T>(rp, (uint32_t)hoff[k]);
                V2<T> v;
                v.rho = r;
                v.psi = (T)psi_signed<double>((double)r, ph);
                (&tile[slot][0][0])[e] = v;
            }
        }
    };

    LanePull L;
    lane_setup<D, T>(g, active ? x : 0, active ? y : 0, L);
    const bool clear = tile_clear<D, TX, TY>(g, t.x0, t.y0);

#pragma unroll 1
    for (int k = 0; k < 4; ++k) load_plane(k, t.m0 - 2 + k);

#pragma unroll 1
    for (int m = t.m0; m < t.m1; ++m) {
        PlanePull P;
        plane_setup<D, T>(g, m, P);
        T f[Q];
        if (active) {
            if (clear && P.mok[0] && P.mok[2]) pull_m<D, T, true>(cur, g.N, L, P, f);
            else pull_m<D, T, false>(cur, g.N, L, P, f);
        }
        load_plane((m - t.m0 + 4) % 5, m + 2);
        __syncthreads();
        if (active) {
            int sl[5];
#pragma unroll
            for (int d = 0; d < 5; ++d) sl[d] = (m - t.m0 + d) % 5;   // plane m + d - 2
            const int hy0 = (D == 3) ? ty + 2 : 0;
            const V2<T> c0 = tile[sl[2]][hy0][tx + 2];
            // force stencils (Sec. 2.3): sums of 3 w_i c_i times
            // [4/3 psi(r+c_i) - 1/6 psi(r+2c_i)] and [rho(r+2c_i) - 2 rho(r+c_i)]
            double G[3] = {0.0, 0.0, 0.0}, K[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
                if (cx == 0 && cy == 0 && cz == 0) continue;
                // 3 w_i: product of one-dimensional weights 2/3 (c=0), 1/6 (c=+-1)
                double w3 = 3.0;
                w3 *= (cx ? 1.0 / 6.0 : 2.0 / 3.0);
                w3 *= (cy ? 1.0 / 6.0 : 2.0 / 3.0);
                if (D == 3) w3 *= (cz ? 1.0 / 6.0 : 2.0 / 3.0);
                V2<T> v1, v2;
                if (D == 3) {
                    v1 = tile[sl[2 + cz]][hy0 + cy][tx + 2 + cx];
                    v2 = tile[sl[2 + 2 * cz]][hy0 + 2 * cy][tx + 2 + 2 * cx];
                } else {
                    v1 = tile[sl[2 + cy]][0][tx + 2 + cx];
                    v2 = tile[sl[2 + 2 * cy]][0][tx + 2 + 2 * cx];
                }
                const double tt = w3 * (4.0 / 3.0 * fabs((double)v1.psi) - 1.0 / 6.0 * fabs((double)v2.psi));
                const double kk = w3 * ((double)v2.rho - 2.0 * (double)v1.rho);
                if (cx > 0) { G[0] += tt; K[0] += kk; }
                if (cx < 0) { G[0] -= tt; K[0] -= kk; }
                if (cy > 0) { G[1] += tt; K[1] += kk; }
                if (cy < 0) { G[1] -= tt; K[1] -= kk; }
                if (cz > 0) { G[2] += tt; K[2] += kk; }
                if (cz < 0) { G[2] -= tt; K[2] -= kk; }
                // evaluate the stencil in groups of directions so that only one
                // group of LDS values (widened to FP64) is live at a time
                if (i % 9 == 8) __builtin_amdgcn_sched_barrier(0);
            }
            double rhoc, j[3];
            moments<D, T, double>(f, rhoc, j);
            const double omega = omega_of<double>(rhoc, ph);
            double F[3] = {0.0, 0.0, 0.0}, Phi[3] = {0.0, 0.0, 0.0};
            const double half_rate = (1.0 - 0.5 * omega) * 0.5;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                F[a] = 2.0 * (double)c0.psi * G[a] + ph.kappa * rhoc * K[a];
                // q_a at r + e_a (source of c_a = -1, index 0) and r - e_a (index 2);
                // behind a wall the mirrored value is the cell itself, negated
                const T* qa = q + (size_t)a * g.N;
                const auto qm0 = plane_rsrc(qa + P.mself, P.bytes);
                const T qself = bld<T>(qm0, L.ip);
                T qp, qm;
                if (a == MA) {
                    qp = P.mok[0] ? bld<T>(plane_rsrc(qa + P.mo[0], P.bytes), L.ip) : -qself;
                    qm = P.mok[2] ? bld<T>(plane_rsrc(qa + P.mo[2], P.bytes), L.ip) : -qself;
                } else if (a == 0) {
                    qp = L.xok[0] ? bld<T>(qm0, L.xo[0] + L.yo[1]) : -qself;
                    qm = L.xok[2] ? bld<T>(qm0, L.xo[2] + L.yo[1]) : -qself;
                } else {
                    qp = L.yok[0] ? bld<T>(qm0, L.xo[1] + L.yo[0]) : -qself;
                    qm = L.yok[2] ? bld<T>(qm0, L.xo[1] + L.yo[2]) : -qself;
                }
                Phi[a] = half_rate * ((double)qp - (double)qm);
            }
            collide<D, T, double>(f, rhoc, j, F, Phi, omega, ph.entropic);
#pragma unroll
            for (int i = 0; i < Q; ++i) bst<T>(plane_rsrc(nxt + (size_t)i * g.N + P.mself, P.bytes), L.ip, f[i]);
        }
        __syncthreads();
    }
}

// Initial velocity shift: the fluid velocity of the exact-difference forcing
// is u + F dt/(2 rho), so starting from a prescribed fluid velocity u0 needs
// the bare velocity u0 - F(rho0)/(2 rho0) in f^eq.  F is the force of
// Sec. 2.3 evaluated on the initial density (FP64, neighbours fetched from
// global memory).  Overwrites u (staged u0) in place; rho is only read.
template <int D>
__global__ __launch_bounds__(256) void k_shift_velocity(const double* __restrict__ rho, double* __restrict__ u,
                                                        Grid g, FlatGrid fg, Phys<double> ph)
{
    constexpr int Q = Lat<D>::Q;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= (uint32_t)g.N) return;
    int co[3];
    flat_coords(cell, fg, co[0], co[1], co[2]);
    auto rho_at = [&](int dx, int dy, int dz) -> double {
        int flip = 0;
        const int x = map_coord(co[0] + dx, g.n[0], g.wall[0], &flip);
        const int y = (D >= 2) ? map_coord(co[1] + dy, g.n[1], g.wall[1], &flip) : 0;
        const int z = (D == 3) ? map_coord(co[2] + dz, g.n[2], g.wall[2], &flip) : 0;
        return rho[x + g.n[0] * y + g.nxny * z];
    };
    const double r0 = rho[cell];
    const double psi0 = psi_signed<double>(r0, ph);
    double G[3] = {0.0, 0.0, 0.0}, K[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
        if (cx == 0 && cy == 0 && cz == 0) continue;
        double w3 = 3.0;
        w3 *= (cx ? 1.0 / 6.0 : 2.0 / 3.0);
        w3 *= (cy ? 1.0 / 6.0 : 2.0 / 3.0);
        if (D == 3) w3 *= (cz ? 1.0 / 6.0 : 2.0 / 3.0);
        const double r1 = rho_at(cx, cy, cz), r2 = rho_at(2 * cx, 2 * cy, 2 * cz);
        const double tt = w3 * (4.0 / 3.0 * fabs(psi_signed<double>(r1, ph)) - 1.0 / 6.0 * fabs(psi_signed<double>(r2, ph)));
        const double kk = w3 * (r2 - 2.0 * r1);
        const int c[3] = {cx, cy, cz};
#pragma unroll
        for (int a = 0; a < D; ++a) {
            if (c[a] > 0) { G[a] += tt; K[a] += kk; }
            if (c[a] < 0) { G[a] -= tt; K[a] -= kk; }
        }
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double F = 2.0 * psi0 * G[a] + ph.kappa * r0 * K[a];
        u[(size_t)a * g.N + cell] -= F / (2.0 * r0);
    }
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ rho0, const double* __restrict__ u0,
                                              T* __restrict__ cur, Grid g, FlatGrid fg)
{
    constexpr int Q = Lat<D>::Q;
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= (uint32_t)g.N) return;
    int co[3];
    flat_coords(cell, fg, co[0], co[1], co[2]);
    const T third = T(1) / T(3);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int c[3] = {cx_<D>(i), cy_<D>(i), cz_<D>(i)};
        // cur_i(x) must pull into f_i(x + c_i) = f^eq_i(x + c_i); if x + c_i is
        // behind a wall it is pulled back into x as direction -i instead.
        int t[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            t[a] = co[a] + c[a];
            if (a >= D) { t[a] = 0; continue; }
            const int n = g.n[a];
            if (!g.wall[a]) t[a] = t[a] < 0 ? t[a] + n : (t[a] >= n ? t[a] - n : t[a]);
            else ok = ok && t[a] >= 0 && t[a] < n;
        }
        int src = cell;
        int dir[3] = {c[0], c[1], c[2]};
        if (ok) {
            src = t[0] + g.n[0] * t[1] + g.nxny * t[2];
        } else {
            dir[0] = -c[0];
            dir[1] = -c[1];
            dir[2] = -c[2];
        }
        const T r = (T)rho0[src];
        T v = r;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const T ua = (T)u0[(size_t)a * g.N + src];
            const T zeta = third + ua * ua;
            v *= (dir[a] == 0) ? (T(1) - zeta) : T(0.5) * (zeta + (dir[a] > 0 ? ua : -ua));
        }
        cur[(size_t)i * g.N + cell] = v;
    }
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_readout(const T* __restrict__ cur, T* __restrict__ rho_out,
                                                 T* __restrict__ u_out, double* __restrict__ partials,
                                                 unsigned* __restrict__ flag, Grid g, FlatGrid fg)
{
    __shared__ double red[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (uint32_t cell = blockIdx.x * 256u + threadIdx.x; cell < (uint32_t)g.N; cell += gridDim.x * 256u) {
        int x, y, z;
        flat_coords(cell, fg, x, y, z);
        PullIdx P;
        pull_setup<D>(g, x, y, z, P);
        T f[Lat<D>::Q];
        pull<D, T>(cur, g, P, f);
        double rho, j[3];
        moments<D, T, double>(f, rho, j);
        rho_out[cell] = (T)rho;
        for (int a = 0; a < D; ++a) u_out[(size_t)a * g.N + cell] = (T)(j[a] / rho);
        acc[0] += rho;
        for (int a = 0; a < D; ++a) acc[1 + a] += j[a];
        if (!(rho > 0.0) || !isfinite(rho)) atomicOr(flag, 1u);
    }
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) partials[blockIdx.x * 4 + threadIdx.x] = red[threadIdx.x][0];
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_pull(const T* __restrict__ cur, T* __restrict__ out, Grid g, FlatGrid fg)
{
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= (uint32_t)g.N) return;
    int x, y, z;
    flat_coords(cell, fg, x, y, z);
    PullIdx P;
    pull_setup<D>(g, x, y, z, P);
    T f[Lat<D>::Q];
    pull<D, T>(cur, g, P, f);
#pragma unroll
    for (int i = 0; i < Lat<D>::Q; ++i) out[(size_t)i * g.N + cell] = f[i];
}

FlatGrid flat_of(const Grid& g)
{
    FlatGrid fg;
    fg.nx = make_fastdiv((uint32_t)g.n[0]);
    fg.ny = make_fastdiv((uint32_t)g.n[1]);
    return fg;
}


template <int D, typename T, int TX, int TY>
hipError_t collide_t(const Launch& L, int tm, const void* cur, void* nxt, const void* rho, const void* q,
                     const Phys<double>& ph)
{
    const Grid& g = L.g;
    const int bx = (g.n[0] + TX - 1) / TX;
    const int by = (D == 3) ? (g.n[1] + TY - 1) / TY : 1;
    const int nm = g.n[D - 1];
    const int bm = (nm + tm - 1) / tm;
    const long long blocks = (long long)bx * by * bm;
    if (blocks <= 0 || blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_collide<D, T, TX, TY>), dim3((unsigned)blocks), dim3(TX, TY), 0, L.stream,
                       (const T*)cur, (T*)nxt, (const T*)rho, (const T*)q, g, ph, bx, by, tm);
    return hipGetLastError();
}

template <int D, typename T>
hipError_t collide_dispatch(const Launch& L, int tx, int ty, int tm, const void* cur, void* nxt,
                            const void* rho, const void* q, const Phys<double>& ph)
{
    if constexpr (D == 2) {
        if (ty != 1) return hipErrorInvalidValue;
        switch (tx) {
        case 64: return collide_t<D, T, 64, 1>(L, tm, cur, nxt, rho, q, ph);
        case 128: return collide_t<D, T, 128, 1>(L, tm, cur, nxt, rho, q, ph);
        case 256: return collide_t<D, T, 256, 1>(L, tm, cur, nxt, rho, q, ph);
        default: return hipErrorInvalidValue;
        }
    } else {
        if (tx == 64 && ty == 4) return collide_t<D, T, 64, 4>(L, tm, cur, nxt, rho, q, ph);
        if (tx == 64 && ty == 2) return collide_t<D, T, 64, 2>(L, tm, cur, nxt, rho, q, ph);
        if (tx == 32 && ty == 8) return collide_t<D, T, 32, 8>(L, tm, cur, nxt, rho, q, ph);
        if (tx == 128 && ty == 2) return collide_t<D, T, 128, 2>(L, tm, cur, nxt, rho, q, ph);
        return hipErrorInvalidValue;
    }
}

unsigned flat_blocks(const Grid& g) { return (unsigned)(((long long)g.N + 255) / 256); }

}  // namespace

bool collide_shape_supported(int D, int tx, int ty)
{
    if (D == 2) return ty == 1 && (tx == 64 || tx == 128 || tx == 256);
    return (tx == 64 && ty == 4) || (tx == 64 && ty == 2) || (tx == 32 && ty == 8) || (tx == 128 && ty == 2);
}

hipError_t launch_macro(const Launch& L, const void* cur, void* rho, void* q, unsigned* flag)
{
    constexpr int TX = 64, TY = 4, TM = 8;
    const Grid& g = L.g;
    const int bx = (g.n[0] + TX - 1) / TX;
    const int by = (L.D == 3) ? (g.n[1] + TY - 1) / TY : 1;
    const int bm = (g.n[L.D - 1] + TM - 1) / TM;
    const unsigned blocks = (unsigned)((long long)bx * by * bm);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_macro<2, float, 256, 1>), dim3((unsigned)((long long)((g.n[0] + 255) / 256) * bm)), dim3(256, 1), 0, L.stream,
                           (const float*)cur, (float*)rho, (float*)q, flag, g, (g.n[0] + 255) / 256, 1, TM);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_macro<2, double, 256, 1>), dim3((unsigned)((long long)((g.n[0] + 255) / 256) * bm)), dim3(256, 1), 0, L.stream,
                           (const double*)cur, (double*)rho, (double*)q, flag, g, (g.n[0] + 255) / 256, 1, TM);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_macro<3, float, TX, TY>), dim3(blocks), dim3(TX, TY), 0, L.stream,
                           (const float*)cur, (float*)rho, (float*)q, flag, g, bx, by, TM);
    else
        hipLaunchKernelGGL((k_macro<3, double, TX, TY>), dim3(blocks), dim3(TX, TY), 0, L.stream,
                           (const double*)cur, (double*)rho, (double*)q, flag, g, bx, by, TM);
    return hipGetLastError();
}

hipError_t launch_collide(const Launch& L, int tx, int ty, int tm, const void* cur, void* nxt,
                          const void* rho, const void* q, const Phys<double>& ph)
{
    if (tm < 1) return hipErrorInvalidValue;
    if (L.D == 2 && !L.fp64) return collide_dispatch<2, float>(L, tx, ty, tm, cur, nxt, rho, q, ph);
    if (L.D == 2) return collide_dispatch<2, double>(L, tx, ty, tm, cur, nxt, rho, q, ph);
    if (!L.fp64) return collide_dispatch<3, float>(L, tx, ty, tm, cur, nxt, rho, q, ph);
    return collide_dispatch<3, double>(L, tx, ty, tm, cur, nxt, rho, q, ph);
}

hipError_t launch_shift_velocity(const Launch& L, const double* rho0, double* u0, const Phys<double>& ph)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2)
        hipLaunchKernelGGL((k_shift_velocity<2>), grid, block, 0, L.stream, rho0, u0, L.g, fg, ph);
    else
        hipLaunchKernelGGL((k_shift_velocity<3>), grid, block, 0, L.stream, rho0, u0, L.g, fg, ph);
    return hipGetLastError();
}

hipError_t launch_init(const Launch& L, const double* rho0, const double* u0, void* cur)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_init<2, float>), grid, block, 0, L.stream, rho0, u0, (float*)cur, L.g, fg);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_init<2, double>), grid, block, 0, L.stream, rho0, u0, (double*)cur, L.g, fg);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_init<3, float>), grid, block, 0, L.stream, rho0, u0, (float*)cur, L.g, fg);
    else
        hipLaunchKernelGGL((k_init<3, double>), grid, block, 0, L.stream, rho0, u0, (double*)cur, L.g, fg);
    return hipGetLastError();
}

hipError_t launch_readout(const Launch& L, const void* cur, void* rho, void* u, double* partials, int nblocks,
                          unsigned* flag)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(nblocks), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_readout<2, float>), grid, block, 0, L.stream, (const float*)cur, (float*)rho, (float*)u, partials, flag, L.g, fg);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_readout<2, double>), grid, block, 0, L.stream, (const double*)cur, (double*)rho, (double*)u, partials, flag, L.g, fg);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_readout<3, float>), grid, block, 0, L.stream, (const float*)cur, (float*)rho, (float*)u, partials, flag, L.g, fg);
    else
        hipLaunchKernelGGL((k_readout<3, double>), grid, block, 0, L.stream, (const double*)cur, (double*)rho, (double*)u, partials, flag, L.g, fg);
    return hipGetLastError();
}

hipError_t launch_pull(const Launch& L, const void* cur, void* out)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_pull<2, float>), grid, block, 0, L.stream, (const float*)cur, (float*)out, L.g, fg);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_pull<2, double>), grid, block, 0, L.stream, (const double*)cur, (double*)out, L.g, fg);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_pull<3, float>), grid, block, 0, L.stream, (const float*)cur, (float*)out, L.g, fg);
    else
        hipLaunchKernelGGL((k_pull<3, double>), grid, block, 0, L.stream, (const double*)cur, (double*)out, L.g, fg);
    return hipGetLastError();
}

}  // namespace elmrt
