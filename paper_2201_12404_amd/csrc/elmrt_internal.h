// elmrt_internal.h -- declarations shared by the C ABI layer and the HIP
// kernels of the library (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/elmrt.h"

#include <string>
#include <stdint.h>

namespace elmrt {

// Each simulation's 256-byte flag block holds the sticky instability flag
// (first 32-bit word) and, at byte 8, a 64-bit count of the cell updates
// whose entropic gamma fell back to 2/omega.
__host__ __device__ inline unsigned long long* gamma_fallbacks(unsigned* flag)
{
    return reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(flag) + 8);
}

// Grid description passed by value to every kernel.
struct Grid {
    int n[3];      // nx, ny, nz (nz = 1 in 2-D)
    int wall[3];   // 1: half-way bounce-back walls at both ends of the axis
    int N;         // number of cells (< 2^31)
    int nxny;
};

// Equation of state and viscosity constants, in working precision.
template <typename T>
struct Phys {
    T RT;          // R T
    T b;           // Peng-Robinson co-volume
    T aal;         // a alpha(T)
    T kappa;       // capillarity kappa~
    T nu_v;        // vapour viscosity
    T dnu;         // nu_l - nu_v
    T rho_v;       // lower density anchor of nu(rho)
    T inv_drho;    // 1 / (rho_l - rho_v), 0 when nu is uniform
    T g[3];        // uniform body acceleration (F gains rho g)
    int entropic;  // 1: entropic gamma, 0: BGK
    int trace_in_h;  // 1: the trace of the second moments is part of h, 0: of s
    int phi_fluid;   // 1: the flux of Phi uses the fluid velocity u + F/(2 rho)
};

// One simulation of a batch: its buffers, grid, constants and tilings, and the
// first workgroup index of its tiles in the batched moment and collision
// launches.  The table lives in device memory; every field is read uniformly.
struct BatchJob {
    const void* buf[2];   // population buffers
    void* rho;
    void* q;
    unsigned* flag;
    Grid g;
    Phys<double> ph;
    int mbx, mby, mtm;    // moment-pass tiling
    int cbx, cby, ctm;    // collision tiling
    int mfirst, cfirst;   // first workgroup of this job in each launch (cfirst: a multiple of 8)
    int cur0;             // buffer holding f at batch parity 0
    int cblocks;          // collision workgroups of this job (its range is padded to a multiple of 8)
};

// Every launcher returns the launch status (hipGetLastError after the launch).
// T is float or double, selected by the 'fp64' flag; D is 2 or 3.
struct Launch {
    int D;
    int fp64;
    Grid g;
    hipStream_t stream;
};

// The instability flag is raised for a non-finite or non-positive density, or
// one at or beyond rho_max = 1/b, the pole of the Peng-Robinson pressure.
// q_momentum: store rho u in q (for launch_flux_fluid) instead of the flux.
hipError_t launch_macro(const Launch& L, const void* cur, void* rho, void* q, unsigned* flag, double rho_max,
                        int q_momentum);

// q := rho v^3 per component, v = (q + F/2) / rho with F the force on the
// density field: the flux of Phi with the fluid velocity (q holds rho u).
hipError_t launch_flux_fluid(const Launch& L, const void* rho, void* q, const Phys<double>& ph);

hipError_t launch_collide(const Launch& L, int tx, int ty, int tm, const void* cur, void* nxt,
                          const void* rho, const void* q, const Phys<double>& ph, unsigned* flag);

// u0 -= F(rho0) / (2 rho0) in place (fluid velocity -> bare velocity).
hipError_t launch_shift_velocity(const Launch& L, const double* rho0, double* u0, const Phys<double>& ph);

// u += F(rho) / (2 rho) in place on working-precision arrays (bare velocity ->
// fluid velocity).
hipError_t launch_fluid_velocity(const Launch& L, const void* rho, void* u, const Phys<double>& ph);

// f := f^eq(rho0, u0) stored so that pull-streaming yields f^eq at every cell.
hipError_t launch_init(const Launch& L, const double* rho0, const double* u0, void* cur);

// rho, u of the current state (working precision; not written when rho is
// NULL), per-block compensated FP64 sums of rho and rho u -- (sum,
// correction) of quantity k of block b at partials[8 b + 2 k], nblocks x 8
// doubles -- and the instability flag (as launch_macro).
hipError_t launch_readout(const Launch& L, const void* cur, void* rho, void* u, double* partials,
                          int nblocks, unsigned* flag, double rho_max);

// Blocks of every read-out reduction, and the devices a process may use.
constexpr int kReadoutBlocks = 1024;
constexpr int kMaxDevices = 64;

// Address, on the current device, of the library's static device scratch for
// the partial sums of one read-out (capacity in blocks of k_readout); looked
// up once per device.
hipError_t readout_scratch(double** out, int* capacity_blocks);

// sums[0..3] = merge of nblocks (sum, correction) pairs of partials, in block
// order; *flag_out = *flag when flag_out is not NULL (device pointers).
hipError_t launch_finish_sums(const double* partials, int nblocks, const unsigned* flag, double* sums,
                              unsigned* flag_out, hipStream_t stream);

// f_i(r, t) = pulled populations, written to out[i*N + cell].
hipError_t launch_pull(const Launch& L, const void* cur, void* out);

// Message returned by elmrt_last_error on this thread.
void set_last_error(const std::string& msg);

// Tile shapes compiled for the collision kernel.
bool collide_shape_supported(int D, int tx, int ty);

// Tiling arithmetic shared by the single and batched launches.
struct Tiling {
    int bx, by, bm, tm;   // tiles along x, y, the marching axis; planes per tile
    long long blocks;
};
Tiling macro_tiling(int D, const Grid& g);
Tiling collide_tiling(int D, const Grid& g, int tx, int ty, int tm);
constexpr int kMacroTX = 256;

// Batched launches over a device job table (jobs sorted by first workgroup).
// All jobs share the lattice, the precision and, for the collision, the tile
// shape (tx, ty); 'blocks' is the total workgroup count of the launch.
hipError_t launch_macro_batch(int D, int fp64, const BatchJob* jobs, int njobs, long long blocks, int parity,
                              hipStream_t stream);
hipError_t launch_collide_batch(int D, int fp64, int tx, int ty, const BatchJob* jobs, int njobs,
                                long long blocks, int parity, hipStream_t stream);

// elmrt_batch_create for a workspace that no kernel has read yet: the job
// table is uploaded without waiting for the members' stream, and the batch
// enqueues its launches directly (no graph).  Used by the request loop.
elmrt_status batch_create_fresh(elmrt_sim* const* sims, int32_t count, void* ws, size_t ws_bytes,
                                elmrt_batch** out);

}  // namespace elmrt
