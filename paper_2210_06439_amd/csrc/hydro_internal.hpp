// hydro_internal.hpp -- internal declarations of the gfx950 hydro library.
//
// Geometry of one subgrid (Sec. II, "Data-Structure": 8^3 cells per leaf by
// default, the size being a compile-time choice; 3 ghost layers per side
// here): (N+6)^3 cells per field, x fastest.  The library is built for
// N = 8 (libhydro.so, every entry point) and N = 16 (libhydro_n16.so, the
// plain stages and the time-integration helpers; the fused kernel is
// written for 8^3 subgrids).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hydro.h"

#ifndef HYDRO_SUBGRID_N
#define HYDRO_SUBGRID_N 8
#endif

namespace hydro {

constexpr int NSUB = HYDRO_SUBGRID_N;   // interior cells per dimension
static_assert(NSUB == 8 || NSUB == 16, "subgrid sizes 8 and 16 are supported");
constexpr int NG = 3;                   // ghost layers
constexpr int NB = NSUB + 2 * NG;       // cells per dimension incl. ghosts
constexpr int NPLANE = NB * NB;         // cells per z-plane
constexpr int NCELL = NB * NB * NB;
constexpr int NINT = NSUB * NSUB * NSUB;
constexpr int QN = NSUB + 2;            // reconstructed cells per dimension: [2, NB-2)
constexpr int QCELL = QN * QN * QN;
constexpr int NFACE = (NSUB + 1) * NSUB * NSUB;   // faces per axis
constexpr int NF_MAX = 11;

// Colella-Woodward (1984) steepening and flattening constants, as recommended
// with the method: eta1, eta2, eps1 and K0 of the contact detector, eps and
// omega1, omega2 of the shock detector.
constexpr double CW_ETA1 = 20.0, CW_ETA2 = 0.05, CW_EPS1 = 0.01, CW_K0 = 0.1;
constexpr double CW_EPS_SHOCK = 0.33, CW_OMEGA1 = 0.75, CW_OMEGA2 = 10.0;

// Kernel-side copy of the call's scalar parameters (passed by value).
struct StepArgs {
    double gamma;
    double de_switch;
    double dt;
    int32_t n_sub;
    int32_t fstride;
    const int64_t *offset;
    const double *h;
    const int32_t *n_species;
    int32_t rate;      // 0: U_out = U + dt L(U); 1: U_out = L(U) on the interior
    int32_t sym;       // symmetric (Kurganov-Tadmor 2000) face speeds
    int32_t vel;       // PPM of the velocities s / rho instead of the momenta
    int32_t steepen;   // Colella-Woodward contact steepening
    int32_t flatten;   // Colella-Woodward flattening
    // Runge-Kutta stage form (U0 non-null): U_out = c0 U0 + c1 (U + dt L(U)),
    // or U0 where dt == 0; dt = clock[1] when clock is non-null, else dt.
    const double *clock;
    const double *U0;
    double c0, c1;
    // per-subgrid output offsets (null: the input offsets)
    const int64_t *out_offset;
    // ghost map (27 source subgrids and mode bits per subgrid, as in
    // hydro_ghost_map): when set, the fused step reads ghost cells from the
    // neighbours' interiors instead of the block's own ghost layers
    const int32_t *gsrc, *gmode;
    // launch shape of the fused step: each subgrid's z sweep in 2^log_parts
    // parts (workgroups), items fetched from a counter when dyn; both need
    // scratch (fused_scratch_bytes), all zero between launches.  unpaired:
    // the batch is known to hold no subgrid without species (the kernel
    // without the paired body serves it)
    int32_t log_parts;
    int32_t dyn;
    int32_t unpaired;
    uint32_t *scratch;
};

// The fused kernel's copy of the same parameters, with the option flags as
// bits: the smaller argument block suits that kernel's code generation (the
// plain kernels keep whole ints, which suit theirs).
struct FusedArgs {
    double gamma;
    double de_switch;
    double dt;
    int32_t n_sub;
    int32_t fstride;
    const int64_t *offset;
    const double *h;
    const int32_t *n_species;
    uint32_t rate : 1;
    uint32_t sym : 1;
    uint32_t vel : 1;
    uint32_t steepen : 1;
    uint32_t flatten : 1;
    const double *clock;
    const double *U0;
    double c0, c1;
    const int64_t *out_offset;
    const int32_t *gsrc, *gmode;
    int32_t log_parts;
    uint32_t dyn : 1;
    uint32_t *scratch;
};

inline FusedArgs fused_args(const StepArgs &a) {
    FusedArgs f;
    f.gamma = a.gamma;
    f.de_switch = a.de_switch;
    f.dt = a.dt;
    f.n_sub = a.n_sub;
    f.fstride = a.fstride;
    f.offset = a.offset;
    f.h = a.h;
    f.n_species = a.n_species;
    f.rate = a.rate ? 1 : 0;
    f.sym = a.sym ? 1 : 0;
    f.vel = a.vel ? 1 : 0;
    f.steepen = a.steepen ? 1 : 0;
    f.flatten = a.flatten ? 1 : 0;
    f.clock = a.clock;
    f.U0 = a.U0;
    f.c0 = a.c0;
    f.c1 = a.c1;
    f.out_offset = a.out_offset;
    f.gsrc = a.gsrc;
    f.gmode = a.gmode;
    f.log_parts = a.log_parts;
    f.dyn = a.dyn ? 1 : 0;
    f.scratch = a.scratch;
    return f;
}

inline StepArgs make_args(const hydro_params *p, const hydro_batch *b) {
    StepArgs a;
    a.gamma = p->gamma;
    a.de_switch = p->de_switch;
    a.dt = p->dt;
    a.n_sub = b->n_sub;
    a.fstride = b->fstride;
    a.offset = b->offset;
    a.h = b->h;
    a.n_species = b->n_species;
    a.rate = 0;
    a.sym = (p->flags & HYDRO_FLAG_KT_SYMMETRIC) ? 1 : 0;
    a.vel = (p->flags & HYDRO_FLAG_VELOCITY) ? 1 : 0;
    a.steepen = (p->flags & HYDRO_FLAG_STEEPEN) ? 1 : 0;
    a.flatten = (p->flags & HYDRO_FLAG_FLATTEN) ? 1 : 0;
    a.clock = nullptr;
    a.U0 = nullptr;
    a.c0 = 0.0;
    a.c1 = 1.0;
    a.out_offset = nullptr;
    a.gsrc = nullptr;
    a.gmode = nullptr;
    a.log_parts = 0;
    a.dyn = 0;
    a.unpaired = 0;
    a.scratch = nullptr;
    return a;
}

// Launch wrappers (each returns hipSuccess or the launch error).
hipError_t launch_plain_reconstruct(const StepArgs &a, const double *U, double *Q,
                                    const int64_t *q_offset, hipStream_t st);
hipError_t launch_plain_flux(const StepArgs &a, const double *Q, const int64_t *q_offset,
                             double *F, const int64_t *f_offset, double *amax,
                             int32_t *status, hipStream_t st);
hipError_t launch_plain_divergence(const StepArgs &a, const double *F, const int64_t *f_offset,
                                   const double *U_in, double *U_out, hipStream_t st);

// Fused step: variant index selects the launch shape.
int fused_variant_count();
const char *fused_variant_name(int v);
// whether a step with a's options in variant v needs scratch, and how many
// bytes it needs for n_sub subgrids (zero-filled before first use; the kernel
// leaves it zero)
bool fused_needs_scratch(const StepArgs &a, int v);
int64_t fused_scratch_bytes(int n_sub);
constexpr int64_t fused_scratch_bytes_for(int64_t n_sub) { return 64 + 16 * n_sub; }
// the launch shape for n_sub subgrids when no tuned choice exists
int fused_default_variant(int n_sub);
// the variant's launch-shape fields of a (log_parts, dyn)
void apply_variant(StepArgs &a, int v);
hipError_t launch_fused_step(const StepArgs &a, const double *U_in, double *U_out,
                             double *amax, int32_t *status, int variant, hipStream_t st);
// Row pitch of the blocks the fused kernel reads and writes (its window's NB
// unless the library steps the 8^3 tiles of larger blocks in place).
int fused_global_pitch();
// The fused step of the 16^3 build (tiles.hip): the 8^3 fused kernel
// (compiled into that library for 8^3 tiles of 16^3 blocks) steps each
// subgrid's eight 8^3 tiles in place, reading their 14^3 windows from the
// block and writing their interiors into the output block.
hipError_t launch_tiled_step(const StepArgs &a, const double *U_in, double *U_out, double *amax,
                             int32_t *status, void *stream);
int64_t tiled_work_bytes(int dev);   // work buffers held on device dev
// Device-resident time integration (evolve.hip).
hipError_t launch_fill_ghosts(int n_sub, int fstride, const int64_t *offset,
                              const int32_t *n_species, const int32_t *src, const int32_t *mode,
                              double *U, int32_t *status, hipStream_t st);
hipError_t launch_cfl_dt(int n_sub, const double *h, const double *amax, double cfl,
                         double t_end, double *clock, hipStream_t st);
hipError_t launch_rk_update(int n_sub, int fstride, const int64_t *offset,
                            const int32_t *n_species, double a, const double *U0, double b,
                            const double *Uk, const double *R, const double *clock, double *Uo,
                            hipStream_t st);
int fused_variant_order(int v);
hipError_t launch_tau_resync(const StepArgs &a, double *U, hipStream_t st);

}  // namespace hydro
