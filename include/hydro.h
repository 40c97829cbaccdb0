/*
 * hydro.h -- C ABI of the MI355X (gfx950) FP64 hydro-step library.
 *
 * The library computes one stage of the finite-volume hydro solver the paper
 * describes in Sec. II ("Solvers"): the `reconstruct` step (piecewise-parabolic
 * values of the evolved variables at 26 quadrature points per cell), the
 * `flux` step (central-upwind Kurganov-Tadmor flux, integrated over each face
 * with the 9-point Newton-Cotes/Simpson rule) and the finite-volume divergence,
 * on batches of 8x8x8 subgrids (Sec. II, "Data-Structure") that each carry 3
 * ghost layers, i.e. 14^3 cells per field.
 *
 * Subgrid size.  The paper's subgrids hold 8^3 cells by default and their
 * size is a compile-time choice (Sec. II, "Data-Structure").  Here too: the
 * library is compiled for N interior cells per dimension, N = 8
 * (libhydro.so) or N = 16 (libhydro_n16.so, compiled with
 * -DHYDRO_SUBGRID_N=16), and hydro_subgrid_n() reports which.  Every size
 * below is written for N = 8; for general N a block has N+6 cells per
 * dimension (fstride >= (N+6)^3), the interior is [3, N+3), Q covers the
 * cells [2, N+4)^3 ((N+2)^3 per direction), and the faces of one axis form a
 * box of (N+1) x N x N.  The N = 16 library provides the plain stages, the
 * entropy-tracer re-sync, the ghost fill, the CFL step size, the stage
 * combination and hydro_step.  The fused kernel maps the 8 x 8 cells of a
 * plane onto one 64-lane wave, so there hydro_step steps each subgrid as the
 * eight 8^3 subgrids that tile it (14^3 windows of the block with their
 * ghosts; the step is local, so their interiors, largest speed and status
 * are the subgrid's): the 8^3 fused kernel, compiled into that library for
 * the 16^3 block's row pitch, reads each window in place and writes its
 * interior into the output block.  The tiles' metadata and per-tile results
 * live in buffers of its own per (device, stream), 256 bytes per subgrid,
 * counted by hydro_workspace_bytes.  Its other fused entry points (hydro_step_variant,
 * hydro_step_io, hydro_step_noalloc, hydro_autotune, hydro_plan_create,
 * hydro_rate, hydro_rk_stage, hydro_rk3_create) return HYDRO_EINVAL.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named U, Q, F, amax, status and every array inside hydro_batch
 *    are DEVICE pointers owned by the caller; `params` and `batch` themselves
 *    are host pointers read during the call.  Nothing is retained after the
 *    call returns, except by hydro_plan_create and hydro_rk3_create (see
 *    there) and the fused step's scratch (see hydro_workspace_bytes).
 *  - Every call enqueues its kernels on `stream` (a hipStream_t; NULL means
 *    the default stream) and returns without synchronising.
 *  - Return value: HYDRO_OK, or a negative HYDRO_E* code; hydro_strerror()
 *    describes the code and, for HYDRO_ELAUNCH, the HIP error.  No C++
 *    exception crosses the ABI.
 *  - Subgrid layout (field-major SoA): field f of subgrid s, cell (i,j,k),
 *    i = x fastest, each index in [0,14), lives at
 *        U[offset[s] + f*fstride + (k*14 + j)*14 + i]
 *    Interior cells have i,j,k in [3,11); the rest are ghosts, filled by the
 *    caller.  Fields f = 0..nf-1, nf = 6 + n_species[s]:
 *        rho, sx, sy, sz, egas, tau, spc_1 .. spc_{n_species}.
 *    fstride >= 2744; 2752 (a multiple of 16 doubles) is recommended.
 *    offset[s] must be a multiple of 2 (16-byte aligned field starts).
 *  - Per-subgrid status word (written when `status` is non-NULL): bit 1 =
 *    rho <= 0 at a quadrature point, bit 2 = p <= 0 there, bit 4 = a
 *    non-finite output, bit 8 = invalid metadata (n_species outside 0..5 or
 *    a negative offset; the subgrid is then skipped and its outputs are not
 *    written).
 *  - Floating point: IEEE binary64 on the vector ALUs; no reduced precision.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    HYDRO_OK = 0,
    HYDRO_EINVAL = -1,   /* null pointer, fstride < 2744, n_sub < 0, misalignment */
    HYDRO_ELAUNCH = -2,  /* a HIP runtime call or kernel launch failed             */
    HYDRO_ENODEV = -3,   /* no gfx950 device is current                            */
    HYDRO_ESCRATCH = -4  /* batch larger than hydro_step_noalloc's fixed scratch     */
};

enum { HYDRO_STATUS_RHO = 1, HYDRO_STATUS_P = 2, HYDRO_STATUS_NONFINITE = 4,
       HYDRO_STATUS_BADMETA = 8 };

/* hydro_params.flags bits.  HYDRO_FLAG_KT_SYMMETRIC: the Kurganov-Tadmor
 * (2000) form of the central flux, one speed for both directions,
 * a = max over the face's points and sides of |u_n| + c (a+ = a, a- = -a):
 * the local Lax-Friedrichs flux.  Without it, the one-sided central-upwind
 * speeds (Kurganov, Noelle, Petrova 2001).  The face speed max(a+, -a-) and
 * hence amax are the same either way. */
enum { HYDRO_FLAG_KT_SYMMETRIC = 1 };

/* HYDRO_FLAG_VELOCITY: reconstruct the velocities instead of the momenta
 * (a variant of the piecewise-parabolic reconstruction of Sec. II,
 * "Solvers", which names the evolved variables).  For the three momentum
 * fields, PPM runs on v = s / rho of the cells along each line, and the
 * momentum at a quadrature point is the density reconstructed at that point
 * times the reconstructed velocity.  All other fields, the flux, the
 * divergence and every layout are unchanged.  Honoured by every entry point
 * that reconstructs: hydro_reconstruct, hydro_step, hydro_step_io,
 * hydro_rate, hydro_rk_stage and the plans and RK3 graphs built from
 * params with the flag. */
enum { HYDRO_FLAG_VELOCITY = 2 };

/* HYDRO_FLAG_STEEPEN, HYDRO_FLAG_FLATTEN: the Colella-Woodward (1984)
 * refinements of the piecewise-parabolic reconstruction, applied to the
 * interface values of each line before the monotonicity constraint.
 *   STEEPEN (density only): near a contact -- the density's second
 *   differences on the two sides of the cell have opposite signs, the
 *   density jump rho_{j+1} - rho_{j-1} exceeds 1% of the smaller density, and
 *   gamma K0 |jump| / min(rho) >= |p_{j+1} - p_{j-1}| / min(p) with K0 = 0.1 --
 *   the interface values move toward the neighbours' linear profiles with the
 *   weight eta = clamp(20 (eta~ - 0.05), 0, 1),
 *   eta~ = -(D_{j+1} - D_{j-1}) / (6 (rho_{j+1} - rho_{j-1})).
 *   FLATTEN (all fields): in a compression along the line (u_{j-1} > u_{j+1},
 *   u the velocity along the line direction) with
 *   |p_{j+1} - p_{j-1}| / min(p) > 0.33, the interface values move toward the
 *   cell value with the weight
 *   clamp(10 ((p_{j+1} - p_{j-1}) / (p_{j+2} - p_{j-2}) - 0.75), 0, 1).
 * Pressures are the cells' own (ideal gas with the dual-energy switch).  The
 * method's extra step that takes the larger flattening weight of the upstream
 * neighbour needs pressures three cells away, beyond the ghost layers of the
 * reconstructed cells; the cell's own weight is used.  Honoured by every
 * entry point that reconstructs, like HYDRO_FLAG_VELOCITY (the fused kernel
 * forms the cell pressures of each line from its field window). */
enum { HYDRO_FLAG_STEEPEN = 4, HYDRO_FLAG_FLATTEN = 8 };

typedef struct {
    double gamma;      /* ratio of specific heats (5/3 for the paper's gas)       */
    double de_switch;  /* dual-energy switch eps: p from tau^gamma where the
                          internal energy E - |s|^2/(2 rho) is below eps * E      */
    double dt;         /* step size of the forward-Euler stage; 0 = speeds only   */
    uint32_t flags;    /* HYDRO_FLAG_* bits; any other bit is HYDRO_EINVAL         */
} hydro_params;

typedef struct {
    int32_t n_sub;              /* number of subgrids (0 is a valid no-op)        */
    int32_t fstride;            /* elements between consecutive fields            */
    const int64_t *offset;      /* device [n_sub]: element offset of field 0      */
    const double *h;            /* device [n_sub]: cell size of the subgrid       */
    const int32_t *n_species;   /* device [n_sub]: passive species, 0..5          */
} hydro_batch;

/*
 * hydro_reconstruct -- PPM reconstruction (Sec. II: the `reconstruct` kernel,
 * piecewise-parabolic values at 26 quadrature points).
 *
 * For every cell c in [2,12)^3, every direction d in {-1,0,1}^3 \ {0} and
 * every field, Q holds the value at the surface point c + d/2, reconstructed
 * by 1-D Colella-Woodward PPM along the line of cell centres c + m d,
 * m = -2..2 (monotonised-central slopes, CW84 monotonicity).
 * Output layout: Q[q_offset[s] + (f*26 + n)*1000 + (k'*10 + j')*10 + i'] with
 * (i',j',k') = c - 2 and n = 9(dz+1) + 3(dy+1) + (dx+1), minus 1 when > 13.
 * q_offset: device [n_sub]; each region holds hydro_q_elems(n_species[s]).
 */
int hydro_reconstruct(const hydro_params *params, const hydro_batch *batch,
                      const double *U, double *Q, const int64_t *q_offset,
                      void *stream);

/*
 * hydro_flux -- central-upwind face flux with Simpson quadrature (Sec. II:
 * the `flux` kernel, Newton-Cotes quadrature; the cited Kurganov-Tadmor
 * finite-volume scheme).
 *
 * For each face between cells c_L and c_L + e_a (c_L from 2 to 10 along a,
 * interior along the other two axes): the 9 surface points of the face carry
 * left states Q(c_L, e_a + t) and right states Q(c_R, -e_a + t); the one-sided
 * speeds a+ = max(0, max u_n + c), a- = min(0, min u_n - c) are taken over all
 * 18 point-sides; the point flux
 *     H = ((a+ F(V_L) - a- F(V_R)) + a+ a- (V_R - V_L)) / (a+ - a-)
 * is averaged with the tensor Simpson weights (1,4,1)x(1,4,1)/36.
 * Output: F[f_offset[s] + (f*3 + a)*576 + idx], idx x-fastest over the face
 * box (extent 9 along a, 8 along the others); amax[s] = max over the subgrid's
 * faces of max(a+, -a-); status[s] as above (may be NULL).
 * q_offset, f_offset: device [n_sub]; F regions hold hydro_f_elems(n_species).
 */
int hydro_flux(const hydro_params *params, const hydro_batch *batch,
               const double *Q, const int64_t *q_offset,
               double *F, const int64_t *f_offset,
               double *amax, int32_t *status, void *stream);

/*
 * hydro_divergence -- finite-volume update (Sec. II: finite volumes):
 *     U_out = U_in - (dt/h) ((dF_x + dF_y) + dF_z)   on the 8^3 interior,
 * dF_a the difference of the averaged fluxes on the two faces of the cell
 * normal to a.  Ghost cells of U_out are not written.  U_out must not alias
 * U_in; both use batch->offset and batch->fstride.
 */
int hydro_divergence(const hydro_params *params, const hydro_batch *batch,
                     const double *F, const int64_t *f_offset,
                     const double *U_in, double *U_out, void *stream);

/*
 * hydro_step -- the fused stage: reconstruct + flux + divergence in one
 * persistent launch over the whole batch, without writing Q or F to memory.
 * Same results as the three calls above up to rounding order (the fused
 * kernel sums the Simpson-weighted terms in a different order).  Writes the
 * interior of U_out, amax[s] and status[s] (may be NULL).  U_out must not
 * alias U_in.  Uses the launch shape chosen by hydro_autotune() for this
 * kind of batch when one was tuned, else the default shape.  With the default
 * options (no velocity reconstruction, steepening or flattening) the same
 * launch sweeps the subgrids without species in a second body, which advances
 * two planes per step on the waves that would carry species; its results are
 * the same bits.
 */
int hydro_step(const hydro_params *params, const hydro_batch *batch,
               const double *U_in, double *U_out, double *amax,
               int32_t *status, void *stream);

/*
 * hydro_step_noalloc -- hydro_step for callers that cannot allocate device
 * memory (code under hipGraph stream capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, launch shape and results (bit for
 * bit) as hydro_step, but it never allocates: the scratch of the split and
 * dynamic launch shapes is a fixed array in the library's device code, one
 * per GPU, sized for HYDRO_NOALLOC_MAX_SUB subgrids (about 1 MiB) and held
 * until the process ends.  A batch of more subgrids returns HYDRO_ESCRATCH.
 * Every call on one GPU shares that GPU's array: the call clears the part it
 * uses with a kernel on `stream` first, and calls whose launches overlap on
 * one GPU (on different streams, or in different plans replayed at once)
 * race on it -- serialise them.
 */
#define HYDRO_NOALLOC_MAX_SUB 65536
int hydro_step_noalloc(const hydro_params *params, const hydro_batch *batch,
                       const double *U_in, double *U_out, double *amax,
                       int32_t *status, void *stream);

/*
 * hydro_step_io -- hydro_step with a separate output offset per subgrid:
 * subgrid s is read at batch->offset[s] of U_in and its interior written at
 * out_offset[s] of U_out (device [n_sub], same alignment rule as offset).
 * U_in and U_out may be the same buffer when no subgrid's output region
 * overlaps any subgrid's input region (the caller's responsibility: the
 * library does not check the device arrays for overlap).  This is how a
 * ping-pong pool advances subgrids in both directions in one launch.
 */
int hydro_step_io(const hydro_params *params, const hydro_batch *batch,
                  const int64_t *out_offset, const double *U_in, double *U_out,
                  double *amax, int32_t *status, void *stream);

/*
 * hydro_copy_blocks -- n row copies between device buffers whose rows are
 * row_elems doubles each: row src_row[i] of src (a buffer of src_rows rows)
 * is read once and written to row dst_row0[i] and, when dst_row1 is not
 * NULL, row dst_row1[i] of dst (dst_rows rows).  This is how a serving loop
 * moves new requests' subgrids (Sec. II, "Data-Structure": subgrids with
 * their ghost layers; in this library's layout each is one contiguous block)
 * from a resident catalogue into both copies of their pool slots.  src_row, dst_row0 and dst_row1 are
 * device arrays of n int64.  A pair whose source index lies outside
 * [0, src_rows) writes nothing; a destination index outside [0, dst_rows) is
 * not written.  Destination rows must not overlap source rows and no two
 * pairs may write the same row (neither is checked).  HYDRO_EINVAL for
 * n < 0, row_elems < 1, negative row counts, n * ceil(row_elems / 2048) above
 * 2^31 - 1, or a null src, dst, src_row or dst_row0 when n > 0.  Asynchronous
 * on `stream`.
 */
int hydro_copy_blocks(const double *src, int64_t src_rows, const int64_t *src_row,
                      double *dst, int64_t dst_rows, const int64_t *dst_row0,
                      const int64_t *dst_row1, int n, int64_t row_elems, void *stream);

/* Element counts of one subgrid's Q and F regions: 26*nf*1000 and 3*nf*576
 * (26*nf*(N+2)^3 and 3*nf*(N+1)*N*N for subgrid size N). */
int64_t hydro_q_elems(int n_species);
int64_t hydro_f_elems(int n_species);

/* The subgrid size N this library was compiled for (8 or 16). */
int hydro_subgrid_n(void);

/* Text for a return code (static storage; HIP detail for HYDRO_ELAUNCH). */
const char *hydro_strerror(int code);

/* Device memory the library holds between calls on the current device, in
 * bytes.  The fused step's split and dynamic launch shapes (below) keep
 * per-subgrid partial results and work counters in scratch: 64 + 16 n_sub
 * bytes, zero between launches.  The eager entry points (hydro_step,
 * hydro_step_variant, hydro_step_io, hydro_step_gather, hydro_rate,
 * hydro_rk_stage, hydro_autotune) use one such buffer per (device, stream),
 * allocated (hipMalloc, synchronously zero-filled) the first time a launch on
 * that stream needs it, for at least 65536 subgrids (about 1 MiB), and grown
 * (to at least twice its size, after synchronizing the stream) only when a
 * larger batch needs more, so that first call must not be made while the
 * stream is being captured; launches
 * on one stream run in order and share it.  Plans and RK3 graphs allocate
 * their own at creation and free it when destroyed.  Every other buffer
 * (the unfused form's Q and F, the time integration's work buffers) belongs
 * to the caller.  0 on a host without a GPU. */
int64_t hydro_workspace_bytes(void);

/* ---------------------------------------------------------------------------
 * Launch variants and the autotuner.  The fused step has several launch
 * shapes; all of them compute bitwise-identical results:
 *   0 persistent-1x          one workgroup per CU, subgrids in a static stride
 *   1 persistent-2x          two per CU (the second wave evens out the tail)
 *   2 one-per-subgrid        one workgroup per subgrid
 *   3 persistent-1x-rev      as 0, subgrids in reverse order
 *   4 persistent-1x-dynamic  as 0, each workgroup fetching its next subgrid
 *                            from a counter (scratch)
 *   5, 6, 7 split-2/4/8      each subgrid's sweep along z cut into 2, 4 or 8
 *                            parts of 4, 2 or 1 interior planes, one
 *                            workgroup each; a part also computes the z face
 *                            below and above its planes, in the same
 *                            arithmetic as a whole sweep, and the last part
 *                            to finish combines the subgrid's amax and
 *                            status words (scratch).  More work in all, but
 *                            a batch of fewer subgrids than CUs runs on more
 *                            of the chip (one subgrid: 141 us whole, 36 us in
 *                            8 parts, on an MI355X).
 */

/* Number of launch variants of the fused step, and a short name for each. */
int hydro_variant_count(void);
const char *hydro_variant_name(int variant);

/* hydro_step with an explicit variant (0 .. hydro_variant_count()-1). */
int hydro_step_variant(const hydro_params *params, const hydro_batch *batch,
                       const double *U_in, double *U_out, double *amax,
                       int32_t *status, int variant, void *stream);

/*
 * hydro_autotune -- times every variant on this batch (`reps` launches each,
 * after one warm-up, with HIP events on `stream`, synchronising the stream),
 * records the fastest for batches of this size (keyed by the power-of-two
 * bucket of n_sub) and returns its index, or a
 * negative error code.  times_ms (host, may be NULL) receives
 * hydro_variant_count() mean times.  U_out, amax and status are overwritten.
 */
int hydro_autotune(const hydro_params *params, const hydro_batch *batch,
                   const double *U_in, double *U_out, double *amax,
                   int32_t *status, int reps, float *times_ms, void *stream);

/* The variant hydro_step will use for a batch of n_sub subgrids: the tuned one
 * for that power-of-two bucket, else the default -- the split into P = 1, 2,
 * 4 or 8 parts with the fewest rounds of work items over the CUs, each round
 * weighted by a part's measured time (P = 8 up to 32 subgrids on 256 CUs,
 * P = 4 up to 64, P = 2 up to 128 and for tails such as 300 or 600
 * subgrids), with P = 1 launched as persistent-2x.  max_species is reserved:
 * the choice does not depend on it. */
int hydro_selected_variant(int n_sub, int max_species);

/* ---------------------------------------------------------------------------
 * Captured plans: a fused step recorded once into a hipGraph and replayed.
 * The plan keeps the device pointers and the batch metadata pointers given at
 * creation (not the contents they point to: metadata and field data may be
 * rewritten between replays).  dt can be changed per replay.  The launch
 * shape is the one hydro_selected_variant gives at creation; a split or
 * dynamic shape gets scratch of its own (allocated here, freed by
 * hydro_plan_destroy), so replays of one plan must not overlap each other.
 * Creation reads the species counts once (synchronously): when every subgrid
 * has species the plan launches the kernel without the paired body (which
 * sweeps any subgrid correctly, so counts rewritten later stay correct).
 */
typedef struct hydro_plan hydro_plan;

int hydro_plan_create(const hydro_params *params, const hydro_batch *batch,
                      const double *U_in, double *U_out, double *amax,
                      int32_t *status, void *stream, hydro_plan **plan_out);
int hydro_plan_set_dt(hydro_plan *plan, double dt);
int hydro_plan_launch(hydro_plan *plan, void *stream);
int hydro_plan_destroy(hydro_plan *plan);

/* ---------------------------------------------------------------------------
 * Device-resident time integration.  Sec. V: a time step of the paper's
 * runs holds three hydro iterations (Test 2), and every step determines its
 * step size and exchanges ghost cells (Test 1); ghost handling is a large
 * part of the hydro time on a CPU (Test 3).  The calls below keep all of
 * that on the device: ghost fill from neighbour interiors, a batch-wide CFL
 * reduction that never returns to the host, and the SSP-RK3 combination.
 */

/*
 * Ghost map of a batch: for subgrid s and neighbour direction slot
 * n = 9(dz+1) + 3(dy+1) + (dx+1) (0..26; 13, the subgrid itself, is unused),
 *   src[s*27 + n]  = batch index of the subgrid that holds the source cells of
 *                    the ghosts of s in direction (dx,dy,dz);
 *   mode[s*27 + n] = bit a (1 = x, 2 = y, 4 = z) set where axis a is a
 *                    zero-gradient (outflow) boundary in that direction: the
 *                    source index along a is the nearest interior cell (3 or
 *                    10) of src; clear: the source is the interior cell 8
 *                    cells back along a in src (i - 8*da), i.e. a neighbour or,
 *                    with src = s, a periodic wrap onto itself.
 * Both are device int32 arrays of n_sub*27 entries.
 */
typedef struct {
    const int32_t *src;
    const int32_t *mode;
} hydro_ghost_map;

/*
 * hydro_fill_ghosts -- copies every ghost cell of every subgrid from the
 * interior cell the map names (all fields of the subgrid).  Only interior
 * cells are read and only ghost cells written, so U is updated in place.
 * A map entry naming no valid subgrid, or a source with fewer fields, leaves
 * those ghosts unchanged and sets HYDRO_STATUS_BADMETA in status[s] (status
 * may be NULL; bits are ORed in).
 */
int hydro_fill_ghosts(const hydro_batch *batch, const hydro_ghost_map *map, double *U,
                      int32_t *status, void *stream);

/*
 * hydro_step_gather -- hydro_step whose ghost cells are read through the map
 * instead of from the blocks' own ghost layers: each ghost value is taken, as
 * the fused kernel loads it, from the interior cell that hydro_fill_ghosts
 * would have copied there.  The result equals hydro_fill_ghosts followed by
 * hydro_step bit for bit, without the fill pass and without reading or
 * writing any ghost cell of U_in.  A map entry naming no valid subgrid, or a
 * source with fewer species than the subgrid, is replaced by the subgrid
 * itself with every axis clamped, and HYDRO_STATUS_BADMETA is set in
 * status[s].  The device RK3 graph (hydro_rk3_create) reads its ghosts this
 * way.  U_out must not alias U_in.
 */
int hydro_step_gather(const hydro_params *params, const hydro_batch *batch,
                      const hydro_ghost_map *map, const double *U_in, double *U_out,
                      double *amax, int32_t *status, void *stream);

/*
 * hydro_rate -- the fused stage in rate form: writes R = L(U_in) =
 * -(1/h)((dF_x + dF_y) + dF_z) on the interior of R (same layout as U_in;
 * ghosts of R are not written), amax[s] as hydro_step, and ORs the status
 * bits into status[s] (may be NULL).  params->dt is not used.  R must not
 * alias U_in.
 */
int hydro_rate(const hydro_params *params, const hydro_batch *batch, const double *U_in,
               double *R, double *amax, int32_t *status, void *stream);

/*
 * hydro_cfl_dt -- batch-wide step size on the device:
 *     dt = cfl * min over s with amax[s] > 0 of h[s] / amax[s],
 * cut to t_end - t so that the clock lands exactly on t_end (then t = t_end);
 * dt = 0 once t >= t_end, or when no subgrid has a positive speed and t_end
 * is infinite.  clock: device double[3] = {t, dt, n}, read and updated; n
 * counts the calls that produced dt > 0.
 */
int hydro_cfl_dt(const hydro_batch *batch, const double *amax, double cfl, double t_end,
                 double *clock, void *stream);

/*
 * hydro_tau_resync -- entropy-tracer re-synchronisation after a stage: in
 * every interior cell where the internal energy from the total energy,
 * e_i = E - |s|^2/(2 rho), is reliable (not below params->de_switch * E, the
 * same switch as in the point state), tau is reset to e_i^(1/gamma); other
 * cells and fields are left as they are.  U is updated in place; ghosts are
 * not touched.  params->dt and params->flags are not used.
 */
int hydro_tau_resync(const hydro_params *params, const hydro_batch *batch, double *U,
                     void *stream);

/*
 * hydro_rk_update -- one SSP-RK3 stage combination on the interior:
 *     U_out = a U0 + b (Uk + dt R),  dt = clock[1],
 * or U_out = U0 when dt == 0 (an empty step leaves the state unchanged).
 * U_out may alias U0 or Uk (element-wise update); ghosts are not written.
 */
int hydro_rk_update(const hydro_batch *batch, double a, const double *U0, double b,
                    const double *Uk, const double *R, const double *clock, double *U_out,
                    void *stream);

/*
 * hydro_rk_stage -- a fused Runge-Kutta stage with the step size on the
 * device: U_out = a U0 + b (U_in + dt L(U_in)) on the interior, dt =
 * clock[1], or U_out = U0 where dt == 0.  amax[s] as hydro_step; status bits
 * are ORed into status[s] (may be NULL).  U_out may alias U0 but not U_in.
 */
int hydro_rk_stage(const hydro_params *params, const hydro_batch *batch, const double *U_in,
                   double *U_out, const double *U0, double a, double b, const double *clock,
                   double *amax, int32_t *status, void *stream);

/*
 * SSP-RK3 time steps captured in one hipGraph.  One replay is one step:
 *   R = L(U); clock <- CFL(amax); U1 = U + dt R;
 *   U2 = 3/4 U + 1/4 (U1 + dt L(U1))      (one fused stage);
 *   U  = 1/3 U + 2/3 (U2 + dt L(U2))      (one fused stage).
 * Every L reads its ghost cells through the map, as hydro_step_gather does,
 * so no fill pass runs and no ghost cell of U, U1 or U2 is read or written:
 * U's ghost layers keep whatever they held (call hydro_fill_ghosts to bring
 * them up to date).  U holds the state; U1, U2 and R
 * are work buffers with U's layout; amax [n_sub]; status [n_sub] collects
 * the OR of every stage's bits (clear it before the first step); clock
 * [3] = {t, dt, n} as for hydro_cfl_dt (set t and n before the first step).  Steps past t_end have
 * dt = 0 and leave U unchanged.  The plan keeps every pointer (including
 * batch and map arrays) until destroyed; their contents may change between
 * replays.  A split or dynamic launch shape gets scratch of its own
 * (allocated before the capture, freed by hydro_rk3_destroy); the species
 * counts are read once, as for hydro_plan_create.
 */
typedef struct hydro_rk3 hydro_rk3;

int hydro_rk3_create(const hydro_params *params, const hydro_batch *batch,
                     const hydro_ghost_map *map, double *U, double *U1, double *U2, double *R,
                     double *amax, int32_t *status, double *clock, double cfl, double t_end,
                     void *stream, hydro_rk3 **plan_out);
/* Replays n_steps steps on `stream`. */
int hydro_rk3_launch(hydro_rk3 *plan, int n_steps, void *stream);
int hydro_rk3_destroy(hydro_rk3 *plan);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H */
