// elmrt_kernels.hip -- gfx950 kernels of one time step of the entropic
// multi-relaxation-time two-phase lattice Boltzmann model (Hosseini, Dorschner
// & Karlin, arXiv:2201.12404).
//
// State layout (device): planes normal to the last axis (z in 3-D, y in 2-D)
// are stored one after another, and within a plane the Q populations are
// stored as separate arrays: cur[(m*Q + i)*P + c], m = the plane index, P =
// cells per plane, c = x (+ nx*y in 3-D).  A plane block (Q*P values) is the
// unit a kernel addresses with one scalar resource; population i sits at the
// scalar offset i*P*sizeof(T) in it.  The buffer holds post-collision
// populations f'(r, t-1) at the cell they leave from, so the populations of
// time t are gathered by pulling:
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

#include <mutex>

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

// Number of nonzero components of c_i.
template <int D>
__host__ __device__ constexpr int pair_class(int i)
{
    return (cx_<D>(i) != 0) + (cy_<D>(i) != 0) + (cz_<D>(i) != 0);
}
// The n-th direction of the upper half i > (Q-1)/2 (one per pair (c, -c)),
// ordered by pair_class, then by index.
template <int D>
__host__ __device__ constexpr int stencil_pair(int n)
{
    constexpr int Q = (D == 2) ? 9 : 27;
    for (int k = 1; k <= D; ++k)
        for (int i = (Q + 1) / 2; i < Q; ++i)
            if (pair_class<D>(i) == k && n-- == 0) return i;
    return -1;
}

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

// Cells per plane normal to the last axis.
template <int D>
__host__ __device__ __forceinline__ int plane_cells(const Grid& g)
{
    return D == 3 ? g.nxny : g.n[0];
}

// Element index of population i of cell (in-plane offset c, plane m).
template <int D>
__device__ __forceinline__ size_t sidx(const Grid& g, int i, int c, int m)
{
    constexpr int Q = Lat<D>::Q;
    return ((size_t)m * Q + i) * (size_t)plane_cells<D>(g) + c;
}

// Pull addressing of one cell: in-plane source offsets and the source plane
// per velocity component c (index c + 1), with their validity.
struct PullIdx {
    int off[2][3];    // in-plane axes (x; y in 3-D): element offsets
    int pl[3];        // marching axis: source plane
    bool ok[3][3];
    int cself, mself;
};

template <int D>
__device__ __forceinline__ void pull_setup(const Grid& g, int x, int y, int z, PullIdx& P)
{
    const int co[3] = {x, y, z};
    const int st[2] = {1, g.n[0]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (a >= D) {
                P.ok[a][k] = true;
                if (a < 2) P.off[a][k] = 0;
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
            if (a == D - 1) P.pl[k] = s;
            else P.off[a][k] = s * st[a];
            P.ok[a][k] = ok;
        }
    }
    P.cself = (D == 3) ? x + g.n[0] * y : x;
    P.mself = (D == 3) ? z : y;
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
        const int cm = (D == 3) ? c : b;
        const int src = P.off[0][a] + ((D == 3) ? P.off[1][b] : 0);
        // bounce-back: the population that left r towards the wall, reversed
        const size_t idx = ok ? sidx<D>(g, i, src, P.pl[cm]) : sidx<D>(g, Q - 1 - i, P.cself, P.mself);
        f[i] = cur[idx];
    }
}

// rho = sum f, j = sum c f, accumulated in A in a fixed order (identical
// wherever it is used): differences and sums along x lines, then the line
// sums combined for rho, j_y and j_z.
template <int D, typename T, typename A>
__device__ __forceinline__ void moments(const T (&f)[Lat<D>::Q], A& rho, A (&j)[3])
{
    constexpr int NZ = (D == 3) ? 3 : 1;
    A L[3][3], jx = A(0);
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const int b = 3 * y + 9 * z;
            const A p = (A)f[b + 2], m = (A)f[b], o = (A)f[b + 1];
            jx += p - m;
            L[y][z] = (p + m) + o;
        }
    A r = A(0), jy = A(0), jz = A(0);
#pragma unroll
    for (int z = 0; z < NZ; ++z) {
        r += (L[0][z] + L[1][z]) + L[2][z];
        jy += L[2][z] - L[0][z];
    }
    if (D == 3) {
#pragma unroll
        for (int y = 0; y < 3; ++y) jz += L[y][2] - L[y][0];
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

// Reciprocal and square root: the hardware instructions in FP32 (1 ulp).  In
// FP64 the reciprocal is the hardware estimate refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (the error squares each step: ~1 ulp, against
// ~10 instructions for a correctly rounded division); the square root is
// correctly rounded.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
template <typename T>
__device__ __forceinline__ T root(T x);
template <>
__device__ __forceinline__ float root<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double root<double>(double x) { return sqrt(x); }

// Square root of a normal positive x (or 0) for psi: the hardware reciprocal
// square root estimate y, one Goldschmidt step on (s, h) = (x y, y/2), which
// doubles the correct bits, and one Newton correction of s (error <= 1 ulp;
// the correctly rounded sqrt adds a second correction and denormal scaling).
__device__ __forceinline__ double root_normal(double x)
{
    if (!(x > 0.0)) return 0.0;
    const double y = __builtin_amdgcn_rsq(x);
    double s = x * y, h = 0.5 * y;
    const double r = fma(-s, h, 0.5);
    s = fma(s, r, s);
    h = fma(h, r, h);
    return fma(fma(-s, s, x), h, s);
}

// psi = sqrt(|P - P0|) (Sec. 2.3), P from the Peng-Robinson EOS (Sec. 3.1),
// P0 = rho cs^2; the sign is the sign of the psi term of the force.
template <typename T>
__device__ __forceinline__ T psi_signed(T r, const Phys<T>& ph)
{
    // both terms over one common denominator: one reciprocal
    const T d1 = T(1) - ph.b * r;
    const T d2 = T(1) + T(2) * ph.b * r - ph.b * ph.b * r * r;
    const T P = (r * ph.RT * d2 - ph.aal * r * r * d1) * rcp<T>(d1 * d2);
    const T d = P - r * (T(1) / T(3));
    T s;
    if constexpr (sizeof(T) == 8) s = root_normal(fabs(d));
    else s = root<T>(fabs(d));
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

// Collision of one cell.  f: pulled populations (overwritten with f');
// returns whether the entropic gamma fell back to 2/omega.  Storage is T.  The per-cell scalars (moments, velocity, force terms, Phi,
// omega, the per-axis factors of the product forms) and the large
// per-population terms f^eq and f* are formed in A (FP64); the small terms
// f - f^eq, s, h and the scalar products stay in T; f' is rounded once.  In
// FP32 this keeps the macroscopic fields within ~1e-6 of the FP64 result over
// 1000 steps, where all-FP32 arithmetic drifts by ~5e-5 (low-density
// interface cells, where the bare velocity and F/rho are O(1) and nearly
// cancel, are the most sensitive).
//
// Every product-form quantity is evaluated through its factors: f^eq and f*
// from the x-y factor products times the z factor, the second moments of
// f - f^eq from sums along x lines, and s (the stress part, Appendix A) as
// e_z A(x,y) + phi2_z B(x,y) + phi1_z C(x,y), where A, B, C collect the 1-D
// dual functions of the x and y axes.
template <int D, typename T, typename A>
__device__ __forceinline__ bool collide(T (&f)[Lat<D>::Q], A rho, const A (&j)[3], const A (&F)[3],
                                        const A (&Phi)[3], A omega, int entropic, int trace_in_h)
{
    constexpr int Q = Lat<D>::Q;
    constexpr int ZL = (D == 3) ? 0 : 1, ZH = (D == 3) ? 2 : 1;   // z index range (c_z + 1)
    const A third = A(1) / A(3);
    const A inv_rho = rcp<A>(rho);
    A u[3] = {A(0), A(0), A(0)};
    A e[3][3], gs[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= D) {
            e[a][0] = e[a][2] = A(0);
            e[a][1] = A(1);
            continue;
        }
        u[a] = j[a] * inv_rho;
        const A zeta = third + u[a] * u[a];
        e[a][1] = A(1) - zeta;
        e[a][2] = A(0.5) * (zeta + u[a]);
        e[a][0] = A(0.5) * (zeta - u[a]);
    }
    // pass 1: f - f^eq (f^eq formed in A from rho times its x-y factor
    // product and the z factor; the difference is small).  It follows the
    // moments directly, so that their widened copies of f serve it as well.
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const A re = rho * e[0][x] * e[1][y];
#pragma unroll
            for (int z = ZL; z <= ZH; ++z) {
                const int i = x + 3 * y + 9 * (D == 3 ? z : 0);
                f[i] = (T)((A)f[i] - re * e[2][z]);
            }
        }
    bool pos = rho > A(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a >= D) {
            gs[a][0] = gs[a][2] = A(0);
            gs[a][1] = A(1);
            continue;
        }
        const A xs = u[a] + F[a] * inv_rho;
        const A zs = third + xs * xs + Phi[a] * inv_rho;
        gs[a][1] = A(1) - zs;
        gs[a][2] = A(0.5) * (zs + xs);
        gs[a][0] = A(0.5) * (zs - xs);
        pos = pos && gs[a][0] > A(0) && gs[a][1] > A(0) && gs[a][2] > A(0);
    }
    // second moments of f - f^eq (its mass and momentum vanish, so raw and
    // central moments agree), from sums and differences along x lines
    T Pxx = T(0), Pyy = T(0), Pzz = T(0), Pxy = T(0), Pxz = T(0), Pyz = T(0);
    {
        T X1[3][3], L[3][3];
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int z = ZL; z <= ZH; ++z) {
                const int b = 3 * y + 9 * (D == 3 ? z : 0);
                const T p = f[b + 2], m = f[b], o = f[b + 1];
                const T x2 = p + m;
                X1[y][z] = p - m;
                L[y][z] = x2 + o;
                Pxx += x2;
            }
#pragma unroll
        for (int z = ZL; z <= ZH; ++z) {
            Pxy += X1[2][z] - X1[0][z];
            Pyy += L[2][z] + L[0][z];
        }
        if (D == 3) {
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                Pxz += X1[y][2] - X1[y][0];
                Pzz += L[y][2] + L[y][0];
            }
            Pyz = (L[2][2] - L[2][0]) - (L[0][2] - L[0][0]);
        }
    }
    const T om1 = (T)(A(1) - omega);
    if (!entropic) {
        // BGK: f' = f* + (1 - omega)(f - f^eq)
#pragma unroll
        for (int x = 0; x < 3; ++x)
#pragma unroll
            for (int y = 0; y < 3; ++y) {
                const A rg = rho * gs[0][x] * gs[1][y];
#pragma unroll
                for (int z = ZL; z <= ZH; ++z) {
                    const int i = x + 3 * y + 9 * (D == 3 ? z : 0);
                    f[i] = (T)(rg * gs[2][z] + (A)(om1 * f[i]));
                }
            }
        if constexpr (sizeof(T) < sizeof(A)) conserve_mass<D, T, A>(f, rho);
        return false;
    }
    // trace in h (the default reading): s carries the deviatoric part only;
    // otherwise s takes the whole second-order block
    if (trace_in_h) {
        const T tr = (D == 3) ? (Pxx + Pyy + Pzz) * (T(1) / T(3)) : (Pxx + Pyy) * T(0.5);
        Pxx -= tr;
        Pyy -= tr;
        Pzz = (D == 3) ? Pzz - tr : T(0);
    }
    // 1-D duals: phi0 = the equilibrium factors, phi1 = {u - 1/2, -2u, u + 1/2},
    // phi2 = {1/2, -1, 1/2}
    T ef[3][3], p1[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int k = 0; k < 3; ++k) ef[a][k] = (T)e[a][k];
        p1[a][0] = (T)(u[a] - A(0.5));
        p1[a][1] = (T)(A(-2) * u[a]);
        p1[a][2] = (T)(u[a] + A(0.5));
    }
    const T p2[3] = {T(0.5), T(-1), T(0.5)};
    T s[Q];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const T ex = ef[0][x], ey = ef[1][y], px = p1[0][x], py = p1[1][y];
            const T Axy = (Pxx * p2[x]) * ey + ex * (Pyy * p2[y]) + (Pxy * px) * py;
            if (D == 3) {
                const T Bxy = (Pzz * ex) * ey;
                const T Cxy = (Pxz * px) * ey + ex * (Pyz * py);
#pragma unroll
                for (int z = 0; z < 3; ++z) s[x + 3 * y + 9 * z] = Axy * ef[2][z] + Bxy * p2[z] + Cxy * p1[2][z];
            } else {
                s[x + 3 * y] = Axy;
            }
        }
    // entropic scalar products <s|h> and <h|h> with weights 1/f*
    T ig[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) ig[a][k] = (a >= D) ? T(1) : rcp<T>((T)gs[a][k]);
    const T irt = (T)inv_rho;
    T wxy[3][3];
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) wxy[x][y] = irt * ig[0][x] * ig[1][y];
    // layer by layer in z: the x-y weights inside a layer, the layer's z
    // weight once on its sums
    T S = T(0), H = T(0);
#pragma unroll
    for (int z = ZL; z <= ZH; ++z) {
        T Sl = T(0), Hl = T(0);
#pragma unroll
        for (int y = 0; y < 3; ++y)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const int i = x + 3 * y + 9 * (D == 3 ? z : 0);
                const T h = f[i] - s[i];
                const T hw = h * wxy[x][y];
                Sl += s[i] * hw;
                Hl += h * hw;
                f[i] = h;
            }
        S += Sl * ig[2][z];
        H += Hl * ig[2][z];
    }
    const bool entropic_gamma = pos && (A)H > Eps2<A>::v * rho;
    const T ch = entropic_gamma ? (T)(omega - A(1)) * S * rcp<T>(H) : T(0);
    // f' = f* + (1 - omega) s + (1 - omega gamma/2) h, f* from rho times its
    // x-y factor product and the z factor
#pragma unroll
    for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const A rg = rho * gs[0][x] * gs[1][y];
#pragma unroll
            for (int z = ZL; z <= ZH; ++z) {
                const int i = x + 3 * y + 9 * (D == 3 ? z : 0);
                f[i] = (T)(rg * gs[2][z] + (A)(om1 * s[i] + ch * f[i]));
            }
        }
    if constexpr (sizeof(T) < sizeof(A)) conserve_mass<D, T, A>(f, rho);
    return !entropic_gamma;
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

// Field planes (rho, q: plain [z][y][x] arrays): a workgroup-uniform base
// pointer in scalar registers plus a 32-bit per-lane byte offset, so no 64-bit
// address is formed per lane.  The base is read from the first lane, which
// states its uniformity to the compiler.
__device__ __forceinline__ const char* plane_ptr(const void* base)
{
    const uint64_t v = (uint64_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const char*)(((uint64_t)hi << 32) | lo);
}

template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ T pld(const char* base, uint32_t off)
{
    return *(gptr<const T>)((gptr<const char>)base + off);
}
// STREAM: a non-temporal store, for fields that are read again only after
// far more data than the caches hold has passed
template <typename T, bool STREAM = false>
__device__ __forceinline__ void pst(const char* base, uint32_t off, T v)
{
    const gptr<T> p = (gptr<T>)((gptr<char>)const_cast<char*>(base) + off);
    if constexpr (STREAM) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Population plane blocks: one raw buffer resource per block (4 scalar
// registers), the population selected by the scalar offset i*P*sizeof(T) and
// the cell by a 32-bit per-lane offset.  A block of Q planes is addressed
// with one resource, so a step holds three (the source planes) instead of Q
// 64-bit bases.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void* base, uint32_t bytes)
{
    const char* b = plane_ptr(base);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(b), (short)0, __builtin_amdgcn_readfirstlane((int)bytes),
                                             0x00020000);
}

template <typename T>
__device__ __forceinline__ T bld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
// Buffer stores; POLICY is the cache-policy operand (0: default; kStream:
// the nt bit, for data that is not read again before far more data than the
// caches hold has passed).
constexpr int kStream = 2;
template <typename T, int POLICY = 0>
__device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v)
{
    if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, POLICY);
    } else {
        using u2 = __attribute__((ext_vector_type(2))) uint32_t;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)voff, (int)soff, POLICY);
    }
}

// In-plane pull sources of one lane, source coordinate x - c (c = -1, 0, +1),
// as byte offsets within a plane.
struct LanePull {
    uint32_t xo[3], yo[3];  // yo = 0 in 2-D
    uint32_t okb;           // bit k: x source k inside the grid; bit 3 + k: y source k
                            // (a bit mask in one vector register, not 6 lane masks)
    uint32_t ip;            // the cell itself
};

// Marching-axis sources (uniform over the workgroup).
struct PlanePull {
    int mo[3];            // source plane of component c (index c + 1)
    bool mok[3];
    int m;                // the plane itself
    int stride;           // cells per plane
    uint32_t bytes;       // bytes of one population plane (P * sizeof(T))
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
    bool xok[3], yok[3] = {true, true, true};
    axis_sources(x, g.n[0], g.wall[0], 1, xo, xok);
    if (D == 3) axis_sources(y, g.n[1], g.wall[1], g.n[0], yo, yok);
    L.okb = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) L.okb |= (xok[k] ? 1u << k : 0u) | (yok[k] ? 8u << k : 0u);
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
    P.stride = plane_cells<D>(g);
    axis_sources(m, g.n[MA], g.wall[MA], 1, P.mo, P.mok);
    P.m = m;
    P.bytes = (uint32_t)P.stride * (uint32_t)sizeof(T);
}

// Resource over the plane block of plane m.
template <int D, typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_of(const T* base, const PlanePull& P, int m)
{
    constexpr int Q = Lat<D>::Q;
    return block_rsrc(base + (size_t)m * Q * P.stride, (uint32_t)Q * P.bytes);
}

// The byte size of a population plane, passed through an empty asm statement
// once per plane so that the compiler forms the Q scalar offsets i * bytes
// next to their loads instead of hoisting all of them out of the plane loop.
__device__ __forceinline__ uint32_t opaque(uint32_t v)
{
    asm volatile("" : "+s"(v));
    return v;
}
// The same for a per-lane value, so that conditions derived from it are
// formed where they are used rather than held as lane masks across the loop.
__device__ __forceinline__ uint32_t opaque_v(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Gather f_i(r, t) of one cell.  FAST: no source of this workgroup and plane
// lies behind a wall (no bounce-back selects needed).
template <int D, typename T, bool FAST>
__device__ __forceinline__ void pull_m(const T* __restrict__ cur, const LanePull& L, const PlanePull& P,
                                       T (&f)[Lat<D>::Q])
{
    constexpr int Q = Lat<D>::Q;
    const uint32_t pb = opaque(P.bytes);
    const uint32_t okb = FAST ? 0u : opaque_v(L.okb);
    __amdgpu_buffer_rsrc_t R[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) R[k] = block_of<D, T>(cur, P, P.mo[k]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i) + 1, cy = cy_<D>(i) + 1, cz = cz_<D>(i) + 1;
        const int cm = (D == 3) ? cz : cy;           // component along the marching axis
        const uint32_t off = L.xo[cx] + ((D == 3) ? L.yo[cy] : 0u);
        if (FAST) {
            f[i] = bld<T>(R[cm], off, (uint32_t)i * pb);
        } else {
            const bool ok = ((okb >> cx) & (okb >> (3 + cy)) & 1u) && P.mok[cm];
            // bounce-back: the population that left r towards the wall, reversed.
            // Both loads are issued (each source is inside the grid), so that the
            // per-lane choice selects a value and never a resource.
            const T fs = bld<T>(R[cm], off, (uint32_t)i * pb);
            const T fb = bld<T>(R[1], L.ip, (uint32_t)(Q - 1 - i) * pb);
            f[i] = ok ? fs : fb;
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

// TOP_DOWN: plane blocks in descending order of the workgroup index.
template <int D, int TX, int TY, bool TOP_DOWN = false>
__device__ __forceinline__ TileCoords tile_of(const Grid& g, int b, int bx, int by, int tm)
{
    TileCoords t;
    const int xb = b % bx;
    b /= bx;
    int yb = 0;
    if (D == 3) {
        yb = b % by;
        b /= by;
    }
    if (TOP_DOWN) b = (g.n[D - 1] + tm - 1) / tm - 1 - b;
    t.x0 = xb * TX;
    t.y0 = yb * TY;
    t.m0 = b * tm;
    t.m1 = min(t.m0 + tm, g.n[D - 1]);
    return t;
}

// Moment pass: rho and the Phi flux q_a = rho u_a^3 of every cell.
template <int D, typename T, int TX, int TY>
__device__ __forceinline__ void macro_tile(int b, const T* __restrict__ cur, T* __restrict__ rho_out,
                                           T* __restrict__ q_out, unsigned* __restrict__ flag, const Grid& g,
                                           int bx, int by, int tm, double rho_max, int q_momentum)
{
    constexpr int Q = Lat<D>::Q;
    // top-down: the planes read last are the bottom ones, which the collision
    // pass (bottom-up) reads first, partly from the Infinity Cache (0.6 % off
    // the step on 256^3)
    const TileCoords t = tile_of<D, TX, TY, true>(g, b, bx, by, tm);
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
        if (clear && P.mok[0] && P.mok[2]) pull_m<D, T, true>(cur, L, P, f);
        else pull_m<D, T, false>(cur, L, P, f);
        double rho, j[3];
        moments<D, T, double>(f, rho, j);
        const size_t mself = (size_t)P.m * P.stride;
        // rho and q are read by the collision pass only after the whole
        // population array has streamed through: non-temporal stores (3 % off
        // this pass on 256^3)
        pst<T, true>(plane_ptr(rho_out + mself), L.ip, (T)rho);
        const double inv = rcp<double>(rho);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            // q_momentum: rho u_a, for k_flux_fluid to turn into q once the
            // density field, and with it the force, is complete
            const double ua = j[a] * inv;
            pst<T, true>(plane_ptr(q_out + (size_t)a * g.N + mself), L.ip, (T)(q_momentum ? j[a] : j[a] * ua * ua));
        }
        bad = bad || !(rho > 0.0) || !isfinite(rho) || rho >= rho_max;
    }
    if (bad) atomicOr(flag, 1u);
}

// Moment pass with two cells per lane, (x, x + 1), for FP32 grids that are
// periodic in x with an even width: each population pair comes in one 8-byte
// load (half the load instructions of one cell per lane), the moments of each
// cell are formed exactly as in macro_tile, so the fields are bitwise the
// same.  A pair whose sources wrap around the row (x = 0 pulling from the
// row's end, or x + 1 = nx - 1 pulling from its start) takes two 4-byte
// loads instead, so that no load reaches into the next row's cache lines.
using f32x2 = float __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f32x2 bld2(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(f32x2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

template <int D>
__device__ __forceinline__ void pull_m2_fast(const float* __restrict__ cur, const LanePull& L0, const LanePull& L1,
                                             const PlanePull& P, float (&f0)[Lat<D>::Q], float (&f1)[Lat<D>::Q])
{
    constexpr int Q = Lat<D>::Q;
    const uint32_t pb = opaque(P.bytes);
    __amdgpu_buffer_rsrc_t R[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) R[k] = block_of<D, float>(cur, P, P.mo[k]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = cx_<D>(i) + 1, cy = cy_<D>(i) + 1, cz = cz_<D>(i) + 1;
        const int cm = (D == 3) ? cz : cy;
        const uint32_t yo = (D == 3) ? L0.yo[cy] : 0u;
        const uint32_t o0 = L0.xo[cx] + yo;
        if (cx == 1) {
            const f32x2 v = bld2(R[cm], o0, (uint32_t)i * pb);
            f0[i] = v.x;
            f1[i] = v.y;
        } else {
            const uint32_t o1 = L1.xo[cx] + yo;
            if (o1 == o0 + 4u) {
                const f32x2 v = bld2(R[cm], o0, (uint32_t)i * pb);
                f0[i] = v.x;
                f1[i] = v.y;
            } else {   // wrapping pair: two loads, both inside the row
                f0[i] = bld<float>(R[cm], o0, (uint32_t)i * pb);
                f1[i] = bld<float>(R[cm], o1, (uint32_t)i * pb);
            }
        }
    }
}

template <int D>
__device__ __forceinline__ void macro_tile2(int b, const float* __restrict__ cur, float* __restrict__ rho_out,
                                            float* __restrict__ q_out, unsigned* __restrict__ flag, const Grid& g,
                                            int bx, int by, int tm, double rho_max, int q_momentum)
{
    constexpr int Q = Lat<D>::Q;
    const TileCoords t = tile_of<D, kMacroTX, 1, true>(g, b, bx, by, tm);
    const int x = t.x0 + 2 * (int)threadIdx.x;
    const int y = (D == 3) ? t.y0 : 0;
    if (x >= g.n[0]) return;   // the width is even: x + 1 is inside too
    LanePull L0, L1;
    lane_setup<D, float>(g, x, y, L0);
    lane_setup<D, float>(g, x + 1, y, L1);
    const bool clear = tile_clear<D, kMacroTX, 1>(g, t.x0, t.y0);
    bool bad = false;
#pragma unroll 1
    for (int m = t.m0; m < t.m1; ++m) {
        PlanePull P;
        plane_setup<D, float>(g, m, P);
        float f0[Q], f1[Q];
        if (clear && P.mok[0] && P.mok[2]) {
            pull_m2_fast<D>(cur, L0, L1, P, f0, f1);
        } else {
            pull_m<D, float, false>(cur, L0, P, f0);
            pull_m<D, float, false>(cur, L1, P, f1);
        }
        double rho0, j0[3], rho1, j1[3];
        moments<D, float, double>(f0, rho0, j0);
        moments<D, float, double>(f1, rho1, j1);
        const size_t mself = (size_t)P.m * P.stride;
        // pairs of 8-byte-aligned values (x and the width are even)
        pst<f32x2, true>(plane_ptr(rho_out + mself), L0.ip, f32x2{(float)rho0, (float)rho1});
        const double inv0 = rcp<double>(rho0), inv1 = rcp<double>(rho1);
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double u0 = j0[a] * inv0, u1 = j1[a] * inv1;
            const float q0 = (float)(q_momentum ? j0[a] : j0[a] * u0 * u0);
            const float q1 = (float)(q_momentum ? j1[a] : j1[a] * u1 * u1);
            pst<f32x2, true>(plane_ptr(q_out + (size_t)a * g.N + mself), L0.ip, f32x2{q0, q1});
        }
        bad = bad || !(rho0 > 0.0) || !isfinite(rho0) || rho0 >= rho_max;
        bad = bad || !(rho1 > 0.0) || !isfinite(rho1) || rho1 >= rho_max;
    }
    if (bad) atomicOr(flag, 1u);
}

// Fused stencil + collision pass.
// Occupancy target of the collision kernel: 3 waves per SIMD (<= 168 VGPRs)
// for D3Q27 in FP32, where it lowers the kernel time by ~12% against the
// register allocation the compiler picks unconstrained (2 waves).
template <int D, typename T>
struct CollideWaves {
    static constexpr int v = (D == 3 && sizeof(T) == 4) ? 3 : 1;
};
template <int D, typename T, int TX, int TY>
__device__ __forceinline__ void collide_tile(int b, const T* __restrict__ cur, T* __restrict__ nxt,
                                             const T* __restrict__ rho, const T* __restrict__ q, const Grid& g,
                                             const Phys<double>& ph, int bx, int by, int tm,
                                             unsigned long long* __restrict__ fallbacks)
{
    constexpr int Q = Lat<D>::Q;
    constexpr int HX = TX + 4;
    constexpr int HY = (D == 3) ? TY + 4 : 1;
    constexpr int NT = TX * TY;
    constexpr int NE = (HX * HY + NT - 1) / NT;   // halo entries staged per thread and plane
    constexpr int MA = D - 1;
    // Six plane slots for the five-plane window of the stencils: the plane
    // staged while a slower wave still computes the previous plane goes to
    // the slot that window does not read, so one barrier per plane (after
    // staging) orders every LDS access.
    constexpr int NS = 6;
    __shared__ double tpsi[NS][HY][HX];  // signed psi, FP64
    __shared__ T trho[NS][HY][HX];       // rho as stored (exact in FP64)

    const TileCoords t = tile_of<D, TX, TY>(g, b, bx, by, tm);
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
    // Entries k < NFULL lie inside the halo for every lane; the test of the
    // others is formed where it is used, not held as a lane mask.
    constexpr int NFULL = (HX * HY) / NT;
    auto staged = [&](int k) { return (int)opaque_v((uint32_t)hoff[k]) >= 0; };
    auto fetch_plane = [&](int m, T (&r)[NE]) {
        int dummy = 0;
        const auto Rr = block_rsrc(rho + (size_t)map_coord(m, g.n[MA], g.wall[MA], &dummy) * mstride,
                                   (uint32_t)mstride * (uint32_t)sizeof(T));
#pragma unroll
        for (int k = 0; k < NE; ++k)
            r[k] = (k < NFULL || staged(k)) ? bld<T>(Rr, (uint32_t)hoff[k], 0u) : T(0);
    };
    auto stage_plane = [&](int slot, const T (&r)[NE]) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            if (k < NFULL || staged(k)) {
                const int e = lid + k * NT;
                (&tpsi[slot][0][0])[e] = psi_signed<double>((double)r[k], ph);
                (&trho[slot][0][0])[e] = r[k];
            }
        }
    };
    auto load_plane = [&](int slot, int m) {
        T r[NE];
        fetch_plane(m, r);
        stage_plane(slot, r);
    };

    LanePull L;
    lane_setup<D, T>(g, active ? x : 0, active ? y : 0, L);
    const bool clear = tile_clear<D, TX, TY>(g, t.x0, t.y0);

#pragma unroll 1
    for (int k = 0; k < 4; ++k) load_plane(k, t.m0 - 2 + k);

    // Per plane: the density loads of the plane entering the window go out
    // first (staging waits only for them), then the Q population pulls and the
    // flux loads for Phi; psi is computed and staged while those are in flight.
    // LDS slot of plane m - 2 is (m - m0) mod 6: a rotation counter kept
    // uniform (scalar), so that the slot arithmetic is not done per lane
    int rot = 0;
#pragma unroll 1
    for (int m = t.m0; m < t.m1; ++m) {
        const int r0 = __builtin_amdgcn_readfirstlane(rot);
        rot = (r0 == NS - 1) ? 0 : r0 + 1;
        PlanePull P;
        plane_setup<D, T>(g, m, P);
        T f[Q];
        T qn[3][3];   // q_a at the sources of c_a = -1 (r + e_a), the cell, c_a = +1
        T rn[NE];
        fetch_plane(m + 2, rn);
        if (active) {
            if (clear && P.mok[0] && P.mok[2]) pull_m<D, T, true>(cur, L, P, f);
            else pull_m<D, T, false>(cur, L, P, f);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                // q_a planes as buffer resources: in-plane byte offsets, no
                // 64-bit address arithmetic per load
                const T* qa = q + (size_t)a * g.N;
                const auto Rm = block_rsrc(qa + (size_t)P.m * P.stride, P.bytes);
                if (a == MA) {
                    qn[a][0] = bld<T>(block_rsrc(qa + (size_t)P.mo[0] * P.stride, P.bytes), L.ip, 0u);
                    qn[a][2] = bld<T>(block_rsrc(qa + (size_t)P.mo[2] * P.stride, P.bytes), L.ip, 0u);
                    qn[a][1] = (P.mok[0] && P.mok[2]) ? T(0) : bld<T>(Rm, L.ip, 0u);
                } else {
                    qn[a][0] = (a == 0) ? bld<T>(Rm, L.xo[0] + L.yo[1], 0u) : bld<T>(Rm, L.xo[1] + L.yo[0], 0u);
                    qn[a][2] = (a == 0) ? bld<T>(Rm, L.xo[2] + L.yo[1], 0u) : bld<T>(Rm, L.xo[1] + L.yo[2], 0u);
                    qn[a][1] = clear ? T(0) : bld<T>(Rm, L.ip, 0u);
                }
            }
        }
        stage_plane(r0 + 4 >= NS ? r0 + 4 - NS : r0 + 4, rn);   // plane m + 2
        __syncthreads();
        if (active) {
            // flux differences for Phi, formed as soon as the loads are back so
            // that three values instead of nine stay live through the stencil
            double dq[3] = {0.0, 0.0, 0.0};
            {
                const uint32_t okb = opaque_v(L.okb);
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    bool okp, okm;
                    if (a == MA) {
                        okp = P.mok[0];
                        okm = P.mok[2];
                    } else {
                        okp = (okb >> (3 * a)) & 1u;
                        okm = (okb >> (3 * a + 2)) & 1u;
                    }
                    const T qp = okp ? qn[a][0] : -qn[a][1];
                    const T qm = okm ? qn[a][2] : -qn[a][1];
                    dq[a] = (double)qp - (double)qm;
                }
            }

            int sl[5];
#pragma unroll
            for (int d = 0; d < 5; ++d) sl[d] = (r0 + d >= NS) ? r0 + d - NS : r0 + d;   // plane m + d - 2
            const int hy0 = (D == 3) ? ty + 2 : 0;
            const double c0psi = tpsi[sl[2]][hy0][tx + 2];
            // force stencils (Sec. 2.3): sums of 3 w_i c_i times
            // [4/3 psi(r+c_i) - 1/6 psi(r+2c_i)] and [rho(r+2c_i) - 2 rho(r+c_i)],
            // taken over the pairs (c, -c) so that each pair costs one
            // difference per radius; 3 w_i = 3 (1/6)^k (2/3)^(D-k) for k
            // nonzero components.  The pairs run class by class (k = 1, 2, 3):
            // the weight falls by exactly 4 from one class to the next, so the
            // sums carry the unnormalised terms 8 d1 - d2 and d2 - 2 d1, are
            // scaled by 4 between classes, and take the last class's weight at
            // the end.  psi and its differences are FP64 (at an interface the
            // terms are O(1) and the force is divided by the vapour density);
            // the density differences are formed in the storage precision,
            // whose rounding (relative to the difference) is below that of the
            // stored densities themselves, and summed in FP64.
            double G[3] = {0.0, 0.0, 0.0}, K[3] = {0.0, 0.0, 0.0};
            auto psi_at = [&](int d, int oy, int ox) { return fabs(tpsi[sl[d]][oy][ox]); };
            auto rho_at = [&](int d, int oy, int ox) { return trho[sl[d]][oy][ox]; };
#pragma unroll
            for (int n = 0; n < (Q - 1) / 2; ++n) {
                const int i = stencil_pair<D>(n);
                const int cx = cx_<D>(i), cy = cy_<D>(i), cz = cz_<D>(i);
                if (n > 0 && pair_class<D>(i) != pair_class<D>(stencil_pair<D>(n - 1))) {
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        G[a] *= 4.0;
                        K[a] *= 4.0;
                    }
                }
                double d1p, d2p;
                T d1r, d2r;
                if (D == 3) {
                    d1p = psi_at(2 + cz, hy0 + cy, tx + 2 + cx) - psi_at(2 - cz, hy0 - cy, tx + 2 - cx);
                    d2p = psi_at(2 + 2 * cz, hy0 + 2 * cy, tx + 2 + 2 * cx) -
                          psi_at(2 - 2 * cz, hy0 - 2 * cy, tx + 2 - 2 * cx);
                    d1r = rho_at(2 + cz, hy0 + cy, tx + 2 + cx) - rho_at(2 - cz, hy0 - cy, tx + 2 - cx);
                    d2r = rho_at(2 + 2 * cz, hy0 + 2 * cy, tx + 2 + 2 * cx) -
                          rho_at(2 - 2 * cz, hy0 - 2 * cy, tx + 2 - 2 * cx);
                } else {
                    d1p = psi_at(2 + cy, 0, tx + 2 + cx) - psi_at(2 - cy, 0, tx + 2 - cx);
                    d2p = psi_at(2 + 2 * cy, 0, tx + 2 + 2 * cx) - psi_at(2 - 2 * cy, 0, tx + 2 - 2 * cx);
                    d1r = rho_at(2 + cy, 0, tx + 2 + cx) - rho_at(2 - cy, 0, tx + 2 - cx);
                    d2r = rho_at(2 + 2 * cy, 0, tx + 2 + 2 * cx) - rho_at(2 - 2 * cy, 0, tx + 2 - 2 * cx);
                }
                const double tt = fma(8.0, d1p, -d2p);
                const double kk = (double)fma(T(-2), d1r, d2r);   // one rounding, relative to kk
                const int c[3] = {cx, cy, cz};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (c[a] > 0) { G[a] += tt; K[a] += kk; }
                    if (c[a] < 0) { G[a] -= tt; K[a] -= kk; }
                }
                // a few pairs at a time, so that only their LDS values are live:
                // the sums so far are pinned here and later LDS loads may not
                // move above this point
                if (n % 4 == 3)
                    asm volatile("" : "+v"(G[0]), "+v"(G[1]), "+v"(G[2]), "+v"(K[0]), "+v"(K[1]), "+v"(K[2])::"memory");
            }
            double rhoc, j[3];
            moments<D, T, double>(f, rhoc, j);
            const double omega = omega_of<double>(rhoc, ph);
            double F[3] = {0.0, 0.0, 0.0}, Phi[3] = {0.0, 0.0, 0.0};
            const double half_rate = (1.0 - 0.5 * omega) * 0.5;
            // the last class's weight 3 w = 1/72 (D3Q27, k = 3) or 1/12 (D2Q9,
            // k = 2); the psi sum also takes the 1/6 of its unnormalised terms
            constexpr double wl = (D == 3) ? 1.0 / 72.0 : 1.0 / 12.0;
            const double cg = c0psi * (wl / 3.0), ck = ph.kappa * wl * rhoc;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                F[a] = cg * G[a] + ck * K[a] + rhoc * ph.g[a];
                Phi[a] = half_rate * dq[a];
            }
            const bool fell_back = collide<D, T, double>(f, rhoc, j, F, Phi, omega, ph.entropic, ph.trace_in_h);
            // count the cells whose gamma fell back: one atomic per wavefront
            // and plane, only when some lane did
            const unsigned long long fb = __ballot(fell_back);
            if (fb != 0ull && __lane_id() == (unsigned)(__ffsll((long long)fb) - 1))
                atomicAdd(fallbacks, (unsigned long long)__popcll(fb));
            {
                const uint32_t pb = opaque(P.bytes);
                const auto R = block_of<D, T>(nxt, P, P.m);
#pragma unroll
                // the new populations are read again only by the next step,
                // after the whole population array has streamed through: the
                // stores bypass cache retention (2 % off the step on 256^3,
                // mostly in the next moment pass)
                for (int i = 0; i < Q; ++i) bst<T, kStream>(R, L.ip, (uint32_t)i * pb, f[i]);
            }
        }
    }
}

// Tile of workgroup b (of nb, bx x-tiles per row) such that the x-tiles of a
// row run on one XCD in consecutive slots: workgroup b runs on XCD b % 8, so
// slot s = b / 8 of XCD j takes x-tile s % bx of row 8 (s / bx) + j.  The
// boundary cache lines that neighbouring x-tiles share are then fetched into
// one L2.  Rows beyond the last full group of 8 keep the natural order.
__device__ __forceinline__ int row_xcd_order(int b, int nb, int bx)
{
    const int full = ((nb / bx) >> 3) << 3;
    if (b >= bx * full) return b;
    const int s = b >> 3, j = b & 7;
    return (s % bx) + bx * (((s / bx) << 3) + j);
}

// Single-simulation entry points: one workgroup per tile.
template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_macro(const T* __restrict__ cur, T* __restrict__ rho_out,
                                                  T* __restrict__ q_out, unsigned* __restrict__ flag, Grid g,
                                                  int bx, int by, int tm, double rho_max, int q_momentum)
{
    macro_tile<D, T, TX, TY>((int)blockIdx.x, cur, rho_out, q_out, flag, g, bx, by, tm, rho_max, q_momentum);
}

// Two cells per lane: kMacroTX / 2 lanes per 256-cell row (macro_tile2).
template <int D>
__global__ __launch_bounds__(kMacroTX / 2) void k_macro2(const float* __restrict__ cur, float* __restrict__ rho_out,
                                                         float* __restrict__ q_out, unsigned* __restrict__ flag,
                                                         Grid g, int bx, int by, int tm, double rho_max,
                                                         int q_momentum)
{
    macro_tile2<D>((int)blockIdx.x, cur, rho_out, q_out, flag, g, bx, by, tm, rho_max, q_momentum);
}

template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(CollideWaves<D, T>::v))) void k_collide(
    const T* __restrict__ cur, T* __restrict__ nxt, const T* __restrict__ rho, const T* __restrict__ q, Grid g,
    Phys<double> ph, int bx, int by, int tm, unsigned long long* __restrict__ fallbacks)
{
    collide_tile<D, T, TX, TY>(row_xcd_order((int)blockIdx.x, (int)gridDim.x, bx), cur, nxt, rho, q, g, ph, bx, by,
                               tm, fallbacks);
}

// Batched entry points: the workgroups of one launch cover the tiles of every
// job of a batch table, job j owning the launch indices [first_j, first_{j+1}).
// The job of a workgroup is found by binary search over the (uniform) table;
// the state buffer holding f(t) alternates with the step parity.
__device__ __forceinline__ int job_of(const BatchJob* __restrict__ jobs, int njobs, int b, int BatchJob::*first)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].*first <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_macro_batch(const BatchJob* __restrict__ jobs, int njobs, int parity)
{
    const int b = (int)blockIdx.x;
    const int j = job_of(jobs, njobs, b, &BatchJob::mfirst);
    const BatchJob& J = jobs[j];
    macro_tile<D, T, TX, TY>(b - J.mfirst, (const T*)J.buf[J.cur0 ^ parity], (T*)J.rho, (T*)J.q, J.flag, J.g,
                             J.mbx, J.mby, J.mtm, 1.0 / J.ph.b, J.ph.phi_fluid);
}

template <int D, typename T, int TX, int TY>
__global__ __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(CollideWaves<D, T>::v))) void k_collide_batch(
    const BatchJob* __restrict__ jobs, int njobs, int parity)
{
    const int b = (int)blockIdx.x;
    const int j = job_of(jobs, njobs, b, &BatchJob::cfirst);
    const BatchJob& J = jobs[j];
    const int lb = b - J.cfirst;   // J.cfirst is a multiple of 8: lb % 8 is the XCD
    if (lb >= J.cblocks) return;   // padding up to the next job
    collide_tile<D, T, TX, TY>(row_xcd_order(lb, J.cblocks, J.cbx), (const T*)J.buf[J.cur0 ^ parity],
                               (T*)J.buf[J.cur0 ^ parity ^ 1],
                               (const T*)J.rho, (const T*)J.q, J.g, J.ph, J.cbx, J.cby, J.ctm,
                               gamma_fallbacks(J.flag));
}

// Force of Sec. 2.3 (psi and capillary stencils, reading R2, R3) plus the
// body force rho g at cell co, in FP64, neighbours fetched from the density
// field in global memory (ghosts mirrored about wall planes, reading R15).
template <int D, typename T>
__device__ __forceinline__ double force_at(const T* __restrict__ rho, const Grid& g, const int (&co)[3],
                                          const Phys<double>& ph, double (&F)[3])
{
    constexpr int Q = Lat<D>::Q;
    auto rho_at = [&](int dx, int dy, int dz) -> double {
        int flip = 0;
        const int x = map_coord(co[0] + dx, g.n[0], g.wall[0], &flip);
        const int y = (D >= 2) ? map_coord(co[1] + dy, g.n[1], g.wall[1], &flip) : 0;
        const int z = (D == 3) ? map_coord(co[2] + dz, g.n[2], g.wall[2], &flip) : 0;
        return (double)rho[x + g.n[0] * y + g.nxny * z];
    };
    const double r0 = rho_at(0, 0, 0);
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
    for (int a = 0; a < 3; ++a) F[a] = (a < D) ? 2.0 * psi0 * G[a] + ph.kappa * r0 * K[a] + r0 * ph.g[a] : 0.0;
    return r0;
}

// Velocity shift between the bare velocity u = sum c f / rho and the fluid
// velocity u + F dt/(2 rho) of the exact-difference forcing: u += sign F/(2 rho)
// in place, F the force on the density field (force_at).  sign = -1 turns a
// prescribed initial fluid velocity into the bare velocity of f^eq; sign = +1
// turns a read-out bare velocity into the fluid velocity.  rho is only read.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_shift_velocity(const T* __restrict__ rho, T* __restrict__ u, Grid g,
                                                        FlatGrid fg, Phys<double> ph, double sign)
{
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= (uint32_t)g.N) return;
    int co[3];
    flat_coords(cell, fg, co[0], co[1], co[2]);
    double F[3];
    const double r0 = force_at<D, T>(rho, g, co, ph, F);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T& ua = u[(size_t)a * g.N + cell];
        ua = (T)((double)ua + sign * F[a] / (2.0 * r0));
    }
}

// The flux of Phi with the fluid velocity (reading switch
// ELMRT_READING_PHI_FLUID_VELOCITY): q holds rho u_a from the moment pass and
// becomes q_a = rho v_a^3 with v = u + F/(2 rho), F on the complete density
// field.  In place: cell r reads and writes only its own q.
template <int D, typename T>
__global__ __launch_bounds__(256) void k_flux_fluid(const T* __restrict__ rho, T* __restrict__ q, Grid g,
                                                    FlatGrid fg, Phys<double> ph)
{
    const uint32_t cell = blockIdx.x * 256u + threadIdx.x;
    if (cell >= (uint32_t)g.N) return;
    int co[3];
    flat_coords(cell, fg, co[0], co[1], co[2]);
    double F[3];
    const double r0 = force_at<D, T>(rho, g, co, ph, F);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T& qa = q[(size_t)a * g.N + cell];
        const double v = ((double)qa + 0.5 * F[a]) / r0;
        qa = (T)(r0 * v * v * v);
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
        cur[sidx<D>(g, i, (D == 3) ? co[0] + g.n[0] * co[1] : co[0], (D == 3) ? co[2] : co[1])] = v;
    }
}

// Neumaier's compensated sum: s plus a running correction c for the low-order
// bits that each addition to s loses.  Pairs merge by adding the other sum to
// s and the other correction to c.
struct CSum {
    double s, c;
};

__device__ __forceinline__ void csum_add(CSum& a, double x)
{
    const double t = a.s + x;
    a.c += (fabs(a.s) >= fabs(x)) ? (a.s - t) + x : (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void csum_merge(CSum& a, const CSum& b)
{
    csum_add(a, b.s);
    a.c += b.c;
}

// rho and u of every cell (working precision; skipped when rho_out is NULL),
// and per-block compensated sums of rho and rho u: each thread accumulates
// its cells, the 64 lanes of a wavefront merge by shuffles, and the four
// wavefronts of the block in order; block b writes (sum, correction) of
// quantity k at partials[8 b + 2 k].  The instability flag is raised for a
// non-finite or non-positive density, or one at or beyond 1/b (the pole of
// the Peng-Robinson pressure).
template <int D, typename T>
__global__ __launch_bounds__(256) void k_readout(const T* __restrict__ cur, T* __restrict__ rho_out,
                                                 T* __restrict__ u_out, double* __restrict__ partials,
                                                 unsigned* __restrict__ flag, Grid g, FlatGrid fg, double rho_max)
{
    __shared__ double red[4][4][2];
    CSum acc[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    bool bad = false;
    for (uint32_t cell = blockIdx.x * 256u + threadIdx.x; cell < (uint32_t)g.N; cell += gridDim.x * 256u) {
        int x, y, z;
        flat_coords(cell, fg, x, y, z);
        PullIdx P;
        pull_setup<D>(g, x, y, z, P);
        T f[Lat<D>::Q];
        pull<D, T>(cur, g, P, f);
        double rho, j[3];
        moments<D, T, double>(f, rho, j);
        if (rho_out) {
            rho_out[cell] = (T)rho;
            for (int a = 0; a < D; ++a) u_out[(size_t)a * g.N + cell] = (T)(j[a] / rho);
        }
        csum_add(acc[0], rho);
        for (int a = 0; a < D; ++a) csum_add(acc[1 + a], j[a]);
        bad = bad || !(rho > 0.0) || !isfinite(rho) || rho >= rho_max;
    }
    if (bad) atomicOr(flag, 1u);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            CSum o;
            o.s = __shfl_down(acc[k].s, off, 64);
            o.c = __shfl_down(acc[k].c, off, 64);
            csum_merge(acc[k], o);
        }
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k) {
            red[wave][k][0] = acc[k].s;
            red[wave][k][1] = acc[k].c;
        }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        CSum t = {red[0][k][0], red[0][k][1]};
        for (int w = 1; w < 4; ++w) csum_merge(t, CSum{red[w][k][0], red[w][k][1]});
        partials[blockIdx.x * 8 + 2 * k] = t.s;
        partials[blockIdx.x * 8 + 2 * k + 1] = t.c;
    }
}

// Merge of the per-block (sum, correction) pairs of k_readout, in block
// order, one quantity per thread: sums[k] = the compensated total of quantity
// k; flag_out (if not NULL) receives the instability flag.  The same
// arithmetic, in the same order, as the host merge of elmrt_read_macros.
__global__ __launch_bounds__(64) void k_finish_sums(const double* __restrict__ partials, int nblocks,
                                                    const unsigned* __restrict__ flag, double* __restrict__ sums,
                                                    unsigned* __restrict__ flag_out)
{
    const int k = threadIdx.x;
    if (k < 4) {
        CSum t = {0.0, 0.0};
        for (int b = 0; b < nblocks; ++b) {
            csum_add(t, partials[b * 8 + 2 * k]);
            t.c += partials[b * 8 + 2 * k + 1];
        }
        sums[k] = t.s + t.c;
    }
    if (k == 4 && flag_out) *flag_out = *flag;
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


unsigned flat_blocks(const Grid& g) { return (unsigned)(((long long)g.N + 255) / 256); }

template <int D, typename T, int TX, int TY>
hipError_t collide_t(const Launch& L, int tm, const void* cur, void* nxt, const void* rho, const void* q,
                     const Phys<double>& ph, unsigned* flag)
{
    const Tiling t = collide_tiling(D, L.g, TX, TY, tm);
    if (t.blocks <= 0 || t.blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_collide<D, T, TX, TY>), dim3((unsigned)t.blocks), dim3(TX, TY), 0, L.stream,
                       (const T*)cur, (T*)nxt, (const T*)rho, (const T*)q, L.g, ph, t.bx, t.by, tm,
                       gamma_fallbacks(flag));
    return hipGetLastError();
}

template <int D, typename T, int TX, int TY>
hipError_t collide_batch_t(const BatchJob* jobs, int njobs, long long blocks, int parity, hipStream_t stream)
{
    if (blocks <= 0 || blocks > 0x7fffffffLL || njobs < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_collide_batch<D, T, TX, TY>), dim3((unsigned)blocks), dim3(TX, TY), 0, stream, jobs,
                       njobs, parity);
    return hipGetLastError();
}

// The compiled collision tile shapes, for the single and the batched launch.
template <int D, typename T>
hipError_t collide_dispatch(const Launch& L, int tx, int ty, int tm, const void* cur, void* nxt,
                            const void* rho, const void* q, const Phys<double>& ph, unsigned* flag)
{
    if constexpr (D == 2) {
        if (ty != 1) return hipErrorInvalidValue;
        switch (tx) {
        case 64: return collide_t<D, T, 64, 1>(L, tm, cur, nxt, rho, q, ph, flag);
        case 128: return collide_t<D, T, 128, 1>(L, tm, cur, nxt, rho, q, ph, flag);
        case 256: return collide_t<D, T, 256, 1>(L, tm, cur, nxt, rho, q, ph, flag);
        default: return hipErrorInvalidValue;
        }
    } else {
        if (tx == 64 && ty == 4) return collide_t<D, T, 64, 4>(L, tm, cur, nxt, rho, q, ph, flag);
        if (tx == 64 && ty == 2) return collide_t<D, T, 64, 2>(L, tm, cur, nxt, rho, q, ph, flag);
        if (tx == 32 && ty == 8) return collide_t<D, T, 32, 8>(L, tm, cur, nxt, rho, q, ph, flag);
        if (tx == 128 && ty == 2) return collide_t<D, T, 128, 2>(L, tm, cur, nxt, rho, q, ph, flag);
        return hipErrorInvalidValue;
    }
}

template <int D, typename T>
hipError_t collide_batch_dispatch(int tx, int ty, const BatchJob* jobs, int njobs, long long blocks, int parity,
                                  hipStream_t stream)
{
    if constexpr (D == 2) {
        if (ty != 1) return hipErrorInvalidValue;
        switch (tx) {
        case 64: return collide_batch_t<D, T, 64, 1>(jobs, njobs, blocks, parity, stream);
        case 128: return collide_batch_t<D, T, 128, 1>(jobs, njobs, blocks, parity, stream);
        case 256: return collide_batch_t<D, T, 256, 1>(jobs, njobs, blocks, parity, stream);
        default: return hipErrorInvalidValue;
        }
    } else {
        if (tx == 64 && ty == 4) return collide_batch_t<D, T, 64, 4>(jobs, njobs, blocks, parity, stream);
        if (tx == 64 && ty == 2) return collide_batch_t<D, T, 64, 2>(jobs, njobs, blocks, parity, stream);
        if (tx == 32 && ty == 8) return collide_batch_t<D, T, 32, 8>(jobs, njobs, blocks, parity, stream);
        if (tx == 128 && ty == 2) return collide_batch_t<D, T, 128, 2>(jobs, njobs, blocks, parity, stream);
        return hipErrorInvalidValue;
    }
}

template <int D, typename T>
hipError_t macro_t(const Launch& L, const void* cur, void* rho, void* q, unsigned* flag, double rho_max,
                   int q_momentum)
{
    const Tiling t = macro_tiling(D, L.g);
    if (t.blocks <= 0 || t.blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    if constexpr (sizeof(T) == 4) {
        if (!L.g.wall[0] && L.g.n[0] % 2 == 0) {
            hipLaunchKernelGGL((k_macro2<D>), dim3((unsigned)t.blocks), dim3(kMacroTX / 2, 1), 0, L.stream,
                               (const float*)cur, (float*)rho, (float*)q, flag, L.g, t.bx, t.by, t.tm, rho_max,
                               q_momentum);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_macro<D, T, kMacroTX, 1>), dim3((unsigned)t.blocks), dim3(kMacroTX, 1), 0, L.stream,
                       (const T*)cur, (T*)rho, (T*)q, flag, L.g, t.bx, t.by, t.tm, rho_max, q_momentum);
    return hipGetLastError();
}

template <int D, typename T>
hipError_t macro_batch_t(const BatchJob* jobs, int njobs, long long blocks, int parity, hipStream_t stream)
{
    if (blocks <= 0 || blocks > 0x7fffffffLL || njobs < 1) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((k_macro_batch<D, T, kMacroTX, 1>), dim3((unsigned)blocks), dim3(kMacroTX, 1), 0, stream,
                       jobs, njobs, parity);
    return hipGetLastError();
}

}  // namespace

// Device scratch of the no-allocation read-out (elmrt_read_sums_noalloc): the
// (sum, correction) pairs of the kReadoutBlocks blocks of k_readout, 64 KiB.
// Each device holds its own copy; host code reaches it only through the
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kReadoutBlocks * 8];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t readout_scratch(double** out, int* capacity_blocks)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    *capacity_blocks = kReadoutBlocks;
    return hipSuccess;
}

hipError_t launch_finish_sums(const double* partials, int nblocks, const unsigned* flag, double* sums,
                              unsigned* flag_out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(64), 0, stream, partials, nblocks, flag, sums, flag_out);
    return hipGetLastError();
}

bool collide_shape_supported(int D, int tx, int ty)
{
    if (D == 2) return ty == 1 && (tx == 64 || tx == 128 || tx == 256);
    return (tx == 64 && ty == 4) || (tx == 64 && ty == 2) || (tx == 32 && ty == 8) || (tx == 128 && ty == 2);
}

// The moment pass takes whole rows of up to 256 cells per workgroup: the
// x-shifted pulls of a row then touch only the row's own cache lines (the
// periodic wrap stays in the row), where 64-cell segments share a line with
// the neighbouring segment at each end.  One plane per workgroup: the pass
// reuses nothing between planes, and more, shorter workgroups keep more loads
// in flight (on 256^3 D3Q27 FP32 0.397 ms against 0.420 ms at 4 planes per
// workgroup and 0.433 ms at 8).
Tiling macro_tiling(int D, const Grid& g)
{
    Tiling t;
    t.bx = (g.n[0] + kMacroTX - 1) / kMacroTX;
    t.by = (D == 3) ? g.n[1] : 1;
    t.tm = 1;
    t.bm = g.n[D - 1];
    t.blocks = (long long)t.bx * t.by * t.bm;
    return t;
}

Tiling collide_tiling(int D, const Grid& g, int tx, int ty, int tm)
{
    Tiling t;
    t.bx = (g.n[0] + tx - 1) / tx;
    t.by = (D == 3) ? (g.n[1] + ty - 1) / ty : 1;
    t.tm = tm;
    t.bm = (g.n[D - 1] + tm - 1) / tm;
    t.blocks = (long long)t.bx * t.by * t.bm;
    return t;
}

hipError_t launch_macro(const Launch& L, const void* cur, void* rho, void* q, unsigned* flag, double rho_max,
                        int q_momentum)
{
    if (L.D == 2 && !L.fp64) return macro_t<2, float>(L, cur, rho, q, flag, rho_max, q_momentum);
    if (L.D == 2) return macro_t<2, double>(L, cur, rho, q, flag, rho_max, q_momentum);
    if (!L.fp64) return macro_t<3, float>(L, cur, rho, q, flag, rho_max, q_momentum);
    return macro_t<3, double>(L, cur, rho, q, flag, rho_max, q_momentum);
}

hipError_t launch_flux_fluid(const Launch& L, const void* rho, void* q, const Phys<double>& ph)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_flux_fluid<2, float>), grid, block, 0, L.stream, (const float*)rho, (float*)q, L.g, fg, ph);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_flux_fluid<2, double>), grid, block, 0, L.stream, (const double*)rho, (double*)q, L.g, fg, ph);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_flux_fluid<3, float>), grid, block, 0, L.stream, (const float*)rho, (float*)q, L.g, fg, ph);
    else
        hipLaunchKernelGGL((k_flux_fluid<3, double>), grid, block, 0, L.stream, (const double*)rho, (double*)q, L.g, fg, ph);
    return hipGetLastError();
}

hipError_t launch_collide(const Launch& L, int tx, int ty, int tm, const void* cur, void* nxt,
                          const void* rho, const void* q, const Phys<double>& ph, unsigned* flag)
{
    if (tm < 1) return hipErrorInvalidValue;
    if (L.D == 2 && !L.fp64) return collide_dispatch<2, float>(L, tx, ty, tm, cur, nxt, rho, q, ph, flag);
    if (L.D == 2) return collide_dispatch<2, double>(L, tx, ty, tm, cur, nxt, rho, q, ph, flag);
    if (!L.fp64) return collide_dispatch<3, float>(L, tx, ty, tm, cur, nxt, rho, q, ph, flag);
    return collide_dispatch<3, double>(L, tx, ty, tm, cur, nxt, rho, q, ph, flag);
}

hipError_t launch_macro_batch(int D, int fp64, const BatchJob* jobs, int njobs, long long blocks, int parity,
                              hipStream_t stream)
{
    if (D == 2 && !fp64) return macro_batch_t<2, float>(jobs, njobs, blocks, parity, stream);
    if (D == 2) return macro_batch_t<2, double>(jobs, njobs, blocks, parity, stream);
    if (!fp64) return macro_batch_t<3, float>(jobs, njobs, blocks, parity, stream);
    return macro_batch_t<3, double>(jobs, njobs, blocks, parity, stream);
}

hipError_t launch_collide_batch(int D, int fp64, int tx, int ty, const BatchJob* jobs, int njobs,
                                long long blocks, int parity, hipStream_t stream)
{
    if (D == 2 && !fp64) return collide_batch_dispatch<2, float>(tx, ty, jobs, njobs, blocks, parity, stream);
    if (D == 2) return collide_batch_dispatch<2, double>(tx, ty, jobs, njobs, blocks, parity, stream);
    if (!fp64) return collide_batch_dispatch<3, float>(tx, ty, jobs, njobs, blocks, parity, stream);
    return collide_batch_dispatch<3, double>(tx, ty, jobs, njobs, blocks, parity, stream);
}

hipError_t launch_shift_velocity(const Launch& L, const double* rho0, double* u0, const Phys<double>& ph)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2)
        hipLaunchKernelGGL((k_shift_velocity<2, double>), grid, block, 0, L.stream, rho0, u0, L.g, fg, ph, -1.0);
    else
        hipLaunchKernelGGL((k_shift_velocity<3, double>), grid, block, 0, L.stream, rho0, u0, L.g, fg, ph, -1.0);
    return hipGetLastError();
}

hipError_t launch_fluid_velocity(const Launch& L, const void* rho, void* u, const Phys<double>& ph)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(flat_blocks(L.g)), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_shift_velocity<2, float>), grid, block, 0, L.stream, (const float*)rho, (float*)u, L.g, fg, ph, 1.0);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_shift_velocity<2, double>), grid, block, 0, L.stream, (const double*)rho, (double*)u, L.g, fg, ph, 1.0);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_shift_velocity<3, float>), grid, block, 0, L.stream, (const float*)rho, (float*)u, L.g, fg, ph, 1.0);
    else
        hipLaunchKernelGGL((k_shift_velocity<3, double>), grid, block, 0, L.stream, (const double*)rho, (double*)u, L.g, fg, ph, 1.0);
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
                          unsigned* flag, double rho_max)
{
    const FlatGrid fg = flat_of(L.g);
    const dim3 grid(nblocks), block(256);
    if (L.D == 2 && !L.fp64)
        hipLaunchKernelGGL((k_readout<2, float>), grid, block, 0, L.stream, (const float*)cur, (float*)rho, (float*)u, partials, flag, L.g, fg, rho_max);
    else if (L.D == 2)
        hipLaunchKernelGGL((k_readout<2, double>), grid, block, 0, L.stream, (const double*)cur, (double*)rho, (double*)u, partials, flag, L.g, fg, rho_max);
    else if (!L.fp64)
        hipLaunchKernelGGL((k_readout<3, float>), grid, block, 0, L.stream, (const float*)cur, (float*)rho, (float*)u, partials, flag, L.g, fg, rho_max);
    else
        hipLaunchKernelGGL((k_readout<3, double>), grid, block, 0, L.stream, (const double*)cur, (double*)rho, (double*)u, partials, flag, L.g, fg, rho_max);
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
