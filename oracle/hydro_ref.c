/*
 * hydro_ref.c -- CPU oracle for the finite-volume hydro step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * FP64 definition that the GPU library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant with the GPU path.
 *
 * What it computes (Sec. II, "Solvers"): the hydro solver evolves the
 * inviscid Euler equations with finite volumes; a `reconstruct` step uses the
 * piecewise-parabolic method to compute the evolved variables at 26
 * quadrature points of every cell, and a `flux` step turns those values into
 * face fluxes integrated with Newton-Cotes quadrature (the central-upwind
 * scheme of Kurganov and Tadmor).  The paper names the kernels and the
 * methods but prints no formulas, so the step list below is the textbook
 * reading of each named method:
 *
 *   O1  the 26 directions d in {-1,0,1}^3 \ {0}; the 13 "lines" are the
 *       directions with n(d) = 9(dz+1) + 3(dy+1) + (dx+1) > 13.
 *   O2  Colella-Woodward (1984) PPM along the line of cell centres c + m d,
 *       m = -2..2: monotonised-central slopes, 4th-order interface values,
 *       CW84 monotonicity.  q+ is the value at c + d/2, q- at c - d/2.
 *   O3  ideal-gas state with a dual-energy switch (entropy tracer tau,
 *       tau^gamma = internal energy density).
 *   O4  central-upwind flux with one-sided speeds a+/a- taken per face
 *       over the face's 9 surface points, integrated with the tensor
 *       Simpson (3-point closed Newton-Cotes) rule.
 *   O5  divergence and forward-Euler update of the N^3 interior.
 *
 * Subgrid size (Sec. II, "Data-Structure": 8^3 cells by default, a
 * compile-time choice): REF_N interior cells per dimension, 8 unless the
 * file is compiled with -DREF_N=<n>; 3 ghost layers on each side.
 *   Options: the symmetric-speed (Kurganov-Tadmor 2000) flux, PPM of the
 *   velocities instead of the momenta, Colella-Woodward contact steepening
 *   and flattening, and the re-synchronisation of the entropy tracer from the
 *   total energy after a stage (all outside the paper's description;
 *   variants of the method).
 *
 * Floating point: IEEE binary64, compiled with -ffp-contract=off; every
 * operation is written in the order that is evaluated.
 *
 * Parity pins: every function here is pinned by the CPU tests against
 * closed forms, hand-computed cases, exactness and symmetry invariants,
 * conservation and an exact Riemann solution; none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- the boundary's data contract, restated for the host ---------------- */

typedef struct {
    double gamma;      /* ratio of specific heats                             */
    double de_switch;  /* dual-energy switch: use tau^gamma if e_i < eps * E  */
    double dt;         /* time step of the forward-Euler stage                */
    uint32_t flags;    /* REF_FLAG_* bits                                     */
} hydro_ref_params;

typedef struct {
    int32_t n_sub;              /* number of subgrids                          */
    int32_t fstride;            /* elements between fields of one subgrid      */
    const int64_t *offset;      /* [n_sub] element offset of field 0           */
    const double *h;            /* [n_sub] cell size                           */
    const int32_t *n_species;   /* [n_sub] passive species, 0..5               */
} hydro_ref_batch;

enum { REF_OK = 0, REF_EINVAL = -1 };

/* Kurganov-Tadmor (2000) form of the central flux: one speed for both
 * directions, a = max over the face's points and sides of |u_n| + c, i.e.
 * a+ = a and a- = -a (the face flux becomes the local Lax-Friedrichs one). */
enum { REF_FLAG_KT_SYMMETRIC = 1 };

/* Velocity reconstruction: for the three momentum fields, PPM runs on the
 * cell velocities v = s / rho along the line, and the momentum at a
 * quadrature point is the product of the density reconstructed at that
 * point and the reconstructed velocity.  Every other field is reconstructed
 * as it is. */
enum { REF_FLAG_VELOCITY = 2 };

/* Colella-Woodward (1984) refinements of the interface values, applied
 * before the monotonicity constraint (their Sec. 3 and 4):
 *  - contact steepening (density only): near a contact, where the density
 *    jump is large against the pressure jump and the second differences on
 *    the two sides have opposite signs, the interface values move toward the
 *    linear extrapolations of the neighbouring cells;
 *  - flattening (all fields): in a strong compression the interface values
 *    move toward the cell value.
 * Both need the cell pressures along the line (ideal gas with the
 * dual-energy switch, as at the quadrature points) and, for flattening, the
 * velocity along the line direction. */
enum { REF_FLAG_STEEPEN = 4, REF_FLAG_FLATTEN = 8 };

static const uint32_t REF_FLAGS_KNOWN =
    REF_FLAG_KT_SYMMETRIC | REF_FLAG_VELOCITY | REF_FLAG_STEEPEN | REF_FLAG_FLATTEN;

/* The constants recommended with the method (Colella & Woodward 1984). */
static const double CW_ETA1 = 20.0, CW_ETA2 = 0.05, CW_EPS1 = 0.01, CW_K0 = 0.1;
static const double CW_EPS_SHOCK = 0.33, CW_OMEGA1 = 0.75, CW_OMEGA2 = 10.0;

static int check_params(const hydro_ref_params *prm)
{
    return (prm && (prm->flags & ~REF_FLAGS_KNOWN) == 0) ? REF_OK : REF_EINVAL;
}

#ifndef REF_N
#define REF_N 8          /* interior cells per dimension                        */
#endif
#define NB (REF_N + 6)   /* cells per dimension incl. 3 ghost layers each side */
#define NC (NB * NB * NB)
#define IL 3             /* interior cells are [IL, IH) in each dimension       */
#define IH (3 + REF_N)
#define QN (REF_N + 2)   /* reconstructed cells per dimension: [2, IH + 1)      */
#define QC (QN * QN * QN)
#define NFACE ((REF_N + 1) * REF_N * REF_N)   /* faces per axis                 */

static const int F_RHO = 0, F_SX = 1, F_EGAS = 4, F_TAU = 5;

static int cell_index(int i, int j, int k) { return (k * NB + j) * NB + i; }

/* O1: direction slot of d, 0..25 (the centre n = 13 is skipped). */
static int dir_slot(int dx, int dy, int dz)
{
    int n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
    return n < 13 ? n : n - 1;
}

static int q_index(int f, int slot, int i, int j, int k)
{
    return (f * 26 + slot) * QC + ((k - 2) * QN + (j - 2)) * QN + (i - 2);
}

/* ---- O2: one-dimensional PPM ------------------------------------------- */

/* Monotonised-central limited slope at the middle of (ul, uc, ur). */
static double mc_slope(double ul, double uc, double ur)
{
    double dm = uc - ul;             /* Delta^- */
    double dp = ur - uc;             /* Delta^+ */
    double d = 0.5 * (dp + dm);
    if (dp * dm > 0.0) {
        double lim = fmin(2.0 * fabs(dm), 2.0 * fabs(dp));
        return copysign(fmin(fabs(d), lim), d);
    }
    return 0.0;
}

/*
 * PPM on the five values u[0..4] = u_{-2..2} of one line with the steepening
 * weight eta and the flattening weight flat (both 0 for classic PPM);
 * returns the value at the +half face (q+) and at the -half face (q-) of the
 * middle cell.
 */
static void ppm_core(const double *u, double eta, double flat, double *qp_out, double *qm_out)
{
    const double sixth = 1.0 / 6.0;
    double s_m = mc_slope(u[0], u[1], u[2]);   /* slope at m = -1 */
    double s_0 = mc_slope(u[1], u[2], u[3]);   /* slope at m =  0 */
    double s_p = mc_slope(u[2], u[3], u[4]);   /* slope at m = +1 */
    double u0 = u[2];
    double qp = 0.5 * (u0 + u[3]) - (s_p - s_0) * sixth;
    double qm = 0.5 * (u[1] + u0) - (s_0 - s_m) * sixth;
    if (eta > 0.0) {
        /* steepening: toward the neighbours' linear profiles at the faces */
        double dm = u[1] + 0.5 * s_m;
        double dp = u[3] - 0.5 * s_p;
        qm = qm * (1.0 - eta) + dm * eta;
        qp = qp * (1.0 - eta) + dp * eta;
    }
    if (flat > 0.0) {
        /* flattening: toward the cell value */
        qm = flat * u0 + (1.0 - flat) * qm;
        qp = flat * u0 + (1.0 - flat) * qp;
    }
    if ((qp - u0) * (u0 - qm) <= 0.0) {
        /* u0 is a local extremum: the parabola is flattened */
        qp = u0;
        qm = u0;
    } else {
        double dq = qp - qm;
        double m6 = 6.0 * (u0 - 0.5 * (qm + qp));
        if (dq * m6 > dq * dq) {
            qm = 3.0 * u0 - 2.0 * qp;          /* overshoot near the - face */
        } else if (-(dq * dq) > dq * m6) {
            qp = 3.0 * u0 - 2.0 * qm;          /* overshoot near the + face */
        }
    }
    *qp_out = qp;
    *qm_out = qm;
}

int hydro_ref_ppm1d(const double *u, double *qp_out, double *qm_out)
{
    ppm_core(u, 0.0, 0.0, qp_out, qm_out);
    return REF_OK;
}

/*
 * Steepening weight of the middle cell from the densities rho[0..4] and
 * pressures p[0..4] of the line (rho_{j-2..j+2}).  The second differences
 * D = rho_{m+1} - 2 rho_m + rho_{m-1} at m = j-1 and j+1 must have opposite
 * signs, the density jump rho_{j+1} - rho_{j-1} must exceed eps1 times the
 * smaller density, and the relative density jump times gamma K0 must be at
 * least the relative pressure jump (a contact, not a shock).  Then, on a
 * uniform grid, eta~ = -(D_{j+1} - D_{j-1}) / (6 (rho_{j+1} - rho_{j-1})) and
 * eta = max(0, min(eta1 (eta~ - eta2), 1)).
 */
static double steepen_weight(double gamma, const double *rho, const double *p)
{
    /* each second difference adds its outer pair first: read backwards,
     * the line gives the same two differences, bit for bit, so the weight
     * keeps the scheme's mirror symmetry exactly */
    double d2m = (rho[0] + rho[2]) - 2.0 * rho[1];
    double d2p = (rho[2] + rho[4]) - 2.0 * rho[3];
    double drho = rho[3] - rho[1];
    if (!(d2p * d2m < 0.0)) return 0.0;
    if (!(fabs(drho) - CW_EPS1 * fmin(fabs(rho[3]), fabs(rho[1])) > 0.0)) return 0.0;
    double jump_rho = gamma * CW_K0 * fabs(drho) / fmin(rho[3], rho[1]);
    double jump_p = fabs(p[3] - p[1]) / fmin(p[3], p[1]);
    if (!(jump_rho >= jump_p)) return 0.0;
    double et = -(d2p - d2m) / (6.0 * drho);
    return fmax(0.0, fmin(CW_ETA1 * (et - CW_ETA2), 1.0));
}

/*
 * Flattening weight of the middle cell from the pressures p[0..4] and the
 * velocities un[0..4] along the line direction: nonzero only in a
 * compression (un_{j-1} > un_{j+1}) with a relative pressure jump
 * |p_{j+1} - p_{j-1}| / min(p_{j+1}, p_{j-1}) above eps; then
 * max(0, min(1, omega2 ((p_{j+1} - p_{j-1}) / (p_{j+2} - p_{j-2}) - omega1))),
 * the ratio taken as +inf where p_{j+2} = p_{j-2}.
 * (The method also takes the larger weight of the upstream neighbour; that
 * needs pressures three cells away, beyond the ghost layers of the cells
 * reconstructed here, so the cell's own weight is used.)
 */
static double flatten_weight(const double *p, const double *un)
{
    double dp1 = p[3] - p[1];
    if (!(un[1] - un[3] > 0.0)) return 0.0;
    if (!(fabs(dp1) / fmin(p[3], p[1]) > CW_EPS_SHOCK)) return 0.0;
    double dp2 = p[4] - p[0];
    /* equal outer pressures: the ratio is read as +inf, whichever way the
     * line runs (a quotient by +0 would be +inf one way and -inf the other) */
    double ratio = dp2 != 0.0 ? dp1 / dp2 : INFINITY;
    return fmax(0.0, fmin(1.0, CW_OMEGA2 * (ratio - CW_OMEGA1)));
}

/*
 * One line with the Colella-Woodward options of prm->flags: u[5] are the
 * field's values, rho[5], p[5] and un[5] the densities, pressures and
 * velocities along the line of the same cells; `is_density` enables the
 * steepening.
 */
int hydro_ref_ppm1d_cw(const hydro_ref_params *prm, const double *u, const double *rho,
                       const double *p, const double *un, int is_density,
                       double *qp_out, double *qm_out)
{
    if (!prm || !u || !rho || !p || !un || !qp_out || !qm_out) return REF_EINVAL;
    double eta = 0.0, flat = 0.0;
    if ((prm->flags & REF_FLAG_STEEPEN) && is_density) eta = steepen_weight(prm->gamma, rho, p);
    if (prm->flags & REF_FLAG_FLATTEN) flat = flatten_weight(p, un);
    ppm_core(u, eta, flat, qp_out, qm_out);
    return REF_OK;
}

/* ---- O3: state and physical flux at one quadrature point ---------------- */

typedef struct {
    double un;    /* normal velocity                                          */
    double cs;    /* sound speed                                              */
    double p;     /* pressure                                                 */
} point_state;

/*
 * Primitive state of the nf conserved values V and the physical flux F along
 * `axis`.  Returns the status bits (1: rho <= 0, 2: p <= 0).
 */
static int state_and_flux(const hydro_ref_params *prm, int nf, int axis,
                          const double *V, double *F, point_state *st)
{
    double gamma = prm->gamma;
    double rho = V[F_RHO];
    double r = 1.0 / rho;
    double vx = V[F_SX + 0] * r;
    double vy = V[F_SX + 1] * r;
    double vz = V[F_SX + 2] * r;
    double ek = 0.5 * ((V[F_SX + 0] * vx + V[F_SX + 1] * vy) + V[F_SX + 2] * vz);
    double E = V[F_EGAS];
    double ei = E - ek;
    if (ei < prm->de_switch * E) {
        ei = pow(V[F_TAU], gamma);     /* dual energy: tau^gamma = e_i */
    }
    double p = (gamma - 1.0) * ei;
    double cs = sqrt((gamma * p) * r);
    double un = axis == 0 ? vx : (axis == 1 ? vy : vz);
    int bits = 0;
    if (rho <= 0.0) bits |= 1;
    if (p <= 0.0) bits |= 2;

    if (F) {
        F[F_RHO] = V[F_SX + axis];
        for (int b = 0; b < 3; b++) {
            F[F_SX + b] = V[F_SX + b] * un;
            if (b == axis) F[F_SX + b] = F[F_SX + b] + p;
        }
        F[F_EGAS] = (E + p) * un;
        F[F_TAU] = V[F_TAU] * un;
        for (int f = 6; f < nf; f++) F[f] = V[f] * un;
    }
    st->un = un;
    st->cs = cs;
    st->p = p;
    return bits;
}

int hydro_ref_state_flux(const hydro_ref_params *prm, int nf, int axis,
                         const double *V, double *F, double *un, double *cs,
                         double *p, int32_t *status)
{
    if (!prm || !V || nf < 6 || nf > 11 || axis < 0 || axis > 2) return REF_EINVAL;
    point_state st;
    int bits = state_and_flux(prm, nf, axis, V, F, &st);
    if (un) *un = st.un;
    if (cs) *cs = st.cs;
    if (p) *p = st.p;
    if (status) *status = bits;
    return REF_OK;
}

/* ---- O4: central-upwind flux of one face, tensor Simpson average -------- */

/*
 * VL, VR: [9][nf] states left and right of the face at the tangential
 * offsets t = (tb, tb2), stored at index (tb2 + 1) * 3 + (tb + 1), where b
 * and b2 are the two other axes in increasing order.  Writes the averaged
 * flux Fbar[nf] and the face speed max(a+, -a-).  Returns status bits.
 */
static int face_flux(const hydro_ref_params *prm, int nf, int axis,
                     const double *VL, const double *VR,
                     double *Fbar, double *amax_face)
{
    double FL[9][11], FR[9][11];
    point_state sl[9], sr[9];
    int bits = 0;
    double lam_p = -INFINITY, lam_m = INFINITY;
    for (int t = 0; t < 9; t++) {
        bits |= state_and_flux(prm, nf, axis, VL + t * nf, FL[t], &sl[t]);
        bits |= state_and_flux(prm, nf, axis, VR + t * nf, FR[t], &sr[t]);
        lam_p = fmax(lam_p, fmax(sl[t].un + sl[t].cs, sr[t].un + sr[t].cs));
        lam_m = fmin(lam_m, fmin(sl[t].un - sl[t].cs, sr[t].un - sr[t].cs));
    }
    double ap = fmax(0.0, lam_p);
    double am = fmin(0.0, lam_m);
    if (prm->flags & REF_FLAG_KT_SYMMETRIC) {
        double a = fmax(ap, -am);
        ap = a;
        am = -a;
    }
    double inv = 1.0 / (ap - am);
    double apam = ap * am;

    const double sixth = 1.0 / 6.0;
    const double two_thirds = 4.0 / 6.0;
    for (int f = 0; f < nf; f++) {
        double H[9];
        for (int t = 0; t < 9; t++) {
            double vl = VL[t * nf + f], vr = VR[t * nf + f];
            H[t] = (((ap * FL[t][f]) - (am * FR[t][f])) + (apam * (vr - vl))) * inv;
        }
        double r[3];
        for (int t2 = 0; t2 < 3; t2++) {
            const double *row = H + t2 * 3;       /* row[0]: tb=-1, row[2]: tb=+1 */
            r[t2] = sixth * (row[0] + row[2]) + two_thirds * row[1];
        }
        Fbar[f] = sixth * (r[0] + r[2]) + two_thirds * r[1];
    }
    *amax_face = fmax(ap, -am);
    return bits;
}

int hydro_ref_face(const hydro_ref_params *prm, int nf, int axis,
                   const double *VL, const double *VR, double *Fbar,
                   double *amax_face, int32_t *status)
{
    if (check_params(prm) != REF_OK || !VL || !VR || !Fbar || nf < 6 || nf > 11 || axis < 0 ||
        axis > 2)
        return REF_EINVAL;
    double a = 0.0;
    int bits = face_flux(prm, nf, axis, VL, VR, Fbar, &a);
    if (amax_face) *amax_face = a;
    if (status) *status = bits;
    return REF_OK;
}

/* ---- argument checks ----------------------------------------------------- */

static int check_batch(const hydro_ref_batch *b)
{
    if (!b || b->n_sub < 0 || b->fstride < NC) return REF_EINVAL;
    if (b->n_sub > 0 && (!b->offset || !b->h || !b->n_species)) return REF_EINVAL;
    for (int s = 0; s < b->n_sub; s++) {
        if (b->n_species[s] < 0 || b->n_species[s] > 5) return REF_EINVAL;
        if (b->offset[s] < 0) return REF_EINVAL;
    }
    return REF_OK;
}

/* ---- per-subgrid stages ------------------------------------------------- */

/* Pressure and velocity of one cell, with the point-state formulas of O3. */
static void cell_state(const hydro_ref_params *prm, const double *U, int fstride, int c,
                       double *p, double v[3])
{
    const int64_t fs = fstride;
    double rho = U[F_RHO * fs + c];
    double sx = U[(F_SX + 0) * fs + c], sy = U[(F_SX + 1) * fs + c], sz = U[(F_SX + 2) * fs + c];
    double r = 1.0 / rho;
    v[0] = sx * r;
    v[1] = sy * r;
    v[2] = sz * r;
    double ek = 0.5 * ((sx * v[0] + sy * v[1]) + sz * v[2]);
    double E = U[F_EGAS * fs + c];
    double ei = E - ek;
    if (ei < prm->de_switch * E) ei = pow(U[F_TAU * fs + c], prm->gamma);
    *p = (prm->gamma - 1.0) * ei;
}

/* O2 over one subgrid: Q for cells [2, IH+1)^3, all 26 directions, nf fields.
 * Density is reconstructed first, so that the velocity option can scale the
 * reconstructed velocities by the density at the same point. */
static void reconstruct_subgrid(const hydro_ref_params *prm, const double *U, int fstride,
                                int nf, double *Q)
{
    const uint32_t flags = prm->flags;
    const int cw = (flags & (REF_FLAG_STEEPEN | REF_FLAG_FLATTEN)) != 0;
    const double *Urho = U + (int64_t)F_RHO * fstride;
    for (int f = 0; f < nf; f++) {
        const double *Uf = U + (int64_t)f * fstride;
        int vel = (flags & REF_FLAG_VELOCITY) && f >= F_SX && f < F_SX + 3;
        for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            int n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
            if (n <= 13) continue;                   /* only the 13 lines */
            int sp = dir_slot(dx, dy, dz), sm = dir_slot(-dx, -dy, -dz);
            for (int k = 2; k <= IH; k++)
            for (int j = 2; j <= IH; j++)
            for (int i = 2; i <= IH; i++) {
                double u[5], rho[5], p[5], un[5];
                for (int m = -2; m <= 2; m++) {
                    int c = cell_index(i + m * dx, j + m * dy, k + m * dz);
                    u[m + 2] = vel ? Uf[c] / Urho[c] : Uf[c];
                    if (cw) {
                        double v[3];
                        cell_state(prm, U, fstride, c, &p[m + 2], v);
                        rho[m + 2] = Urho[c];
                        un[m + 2] = (dx * v[0] + dy * v[1]) + dz * v[2];
                    }
                }
                double qp, qm;
                if (cw)
                    hydro_ref_ppm1d_cw(prm, u, rho, p, un, f == F_RHO, &qp, &qm);
                else
                    hydro_ref_ppm1d(u, &qp, &qm);
                if (vel) {
                    qp = Q[q_index(F_RHO, sp, i, j, k)] * qp;
                    qm = Q[q_index(F_RHO, sm, i, j, k)] * qm;
                }
                Q[q_index(f, sp, i, j, k)] = qp;
                Q[q_index(f, sm, i, j, k)] = qm;
            }
        }
    }
}

/* Index of the face with left cell (i,j,k) on `axis` inside its box of
 * (N+1) x N x N faces (extent N+1 along the axis, x fastest). */
static int face_index(int axis, int i, int j, int k)
{
    const int n = REF_N;
    if (axis == 0) return ((k - IL) * n + (j - IL)) * (n + 1) + (i - 2);
    if (axis == 1) return ((k - IL) * (n + 1) + (j - 2)) * n + (i - IL);
    return ((k - 2) * n + (j - IL)) * n + (i - IL);
}

/* O4 over one subgrid: F[f][axis][NFACE] and the subgrid's max face speed. */
static int flux_subgrid(const hydro_ref_params *prm, const double *Q, int nf,
                        double *F, double *amax_out)
{
    int bits = 0;
    double amax = 0.0;
    double VL[9 * 11], VR[9 * 11], Fbar[11];
    for (int axis = 0; axis < 3; axis++) {
        int b = axis == 0 ? 1 : 0;                  /* tangential axes, b < b2 */
        int b2 = axis == 2 ? 1 : 2;
        int lo[3] = {IL, IL, IL}, hi[3] = {IH, IH, IH};
        lo[axis] = 2;                               /* left cells 2..IH-1 */
        for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
        for (int i = lo[0]; i < hi[0]; i++) {
            int cl[3] = {i, j, k};
            int cr[3] = {i, j, k};
            cr[axis] += 1;
            for (int t2 = -1; t2 <= 1; t2++)
            for (int t1 = -1; t1 <= 1; t1++) {
                int dl[3] = {0, 0, 0}, dr[3] = {0, 0, 0};
                dl[axis] = 1;
                dr[axis] = -1;
                dl[b] = t1; dr[b] = t1;
                dl[b2] = t2; dr[b2] = t2;
                int sl = dir_slot(dl[0], dl[1], dl[2]);
                int sr = dir_slot(dr[0], dr[1], dr[2]);
                int t = (t2 + 1) * 3 + (t1 + 1);
                for (int f = 0; f < nf; f++) {
                    VL[t * nf + f] = Q[q_index(f, sl, cl[0], cl[1], cl[2])];
                    VR[t * nf + f] = Q[q_index(f, sr, cr[0], cr[1], cr[2])];
                }
            }
            double af;
            bits |= face_flux(prm, nf, axis, VL, VR, Fbar, &af);
            int fi = face_index(axis, i, j, k);
            for (int f = 0; f < nf; f++) {
                F[(f * 3 + axis) * NFACE + fi] = Fbar[f];
                if (!isfinite(Fbar[f])) bits |= 4;
            }
            amax = fmax(amax, af);
        }
    }
    if (!isfinite(amax)) bits |= 4;
    *amax_out = amax;
    return bits;
}

/* O5 over one subgrid: U_out = U - (dt/h) ((dFx + dFy) + dFz) on [IL,IH)^3. */
static int divergence_subgrid(const double *F, const double *U, double *Uo,
                              int fstride, int nf, double dt, double h)
{
    int bits = 0;
    double lam = dt / h;
    for (int f = 0; f < nf; f++) {
        const double *Uf = U + (int64_t)f * fstride;
        double *Of = Uo + (int64_t)f * fstride;
        for (int k = IL; k < IH; k++)
        for (int j = IL; j < IH; j++)
        for (int i = IL; i < IH; i++) {
            const double *Fx = F + (f * 3 + 0) * NFACE;
            const double *Fy = F + (f * 3 + 1) * NFACE;
            const double *Fz = F + (f * 3 + 2) * NFACE;
            double dfx = Fx[face_index(0, i, j, k)] - Fx[face_index(0, i - 1, j, k)];
            double dfy = Fy[face_index(1, i, j, k)] - Fy[face_index(1, i, j - 1, k)];
            double dfz = Fz[face_index(2, i, j, k)] - Fz[face_index(2, i, j, k - 1)];
            int c = cell_index(i, j, k);
            double v = Uf[c] - lam * ((dfx + dfy) + dfz);
            Of[c] = v;
            if (!isfinite(v)) bits |= 4;
        }
    }
    return bits;
}

/* ---- the four entry points ------------------------------------------------ */

int hydro_ref_subgrid_n(void) { return REF_N; }
int64_t hydro_ref_q_elems(int n_species) { return (int64_t)26 * (6 + n_species) * QC; }
int64_t hydro_ref_f_elems(int n_species) { return (int64_t)3 * (6 + n_species) * NFACE; }

int hydro_ref_reconstruct(const hydro_ref_params *prm, const hydro_ref_batch *b,
                          const double *U, double *Q, const int64_t *q_offset)
{
    if (check_params(prm) != REF_OK || check_batch(b) != REF_OK) return REF_EINVAL;
    if (b->n_sub > 0 && (!U || !Q || !q_offset)) return REF_EINVAL;
    for (int s = 0; s < b->n_sub; s++)
        reconstruct_subgrid(prm, U + b->offset[s], b->fstride, 6 + b->n_species[s],
                            Q + q_offset[s]);
    return REF_OK;
}

int hydro_ref_flux(const hydro_ref_params *prm, const hydro_ref_batch *b,
                   const double *Q, const int64_t *q_offset, double *F,
                   const int64_t *f_offset, double *amax, int32_t *status)
{
    if (check_params(prm) != REF_OK || check_batch(b) != REF_OK) return REF_EINVAL;
    if (b->n_sub > 0 && (!Q || !q_offset || !F || !f_offset || !amax)) return REF_EINVAL;
    for (int s = 0; s < b->n_sub; s++) {
        double a;
        int bits = flux_subgrid(prm, Q + q_offset[s], 6 + b->n_species[s],
                                F + f_offset[s], &a);
        amax[s] = a;
        if (status) status[s] = bits;
    }
    return REF_OK;
}

int hydro_ref_divergence(const hydro_ref_params *prm, const hydro_ref_batch *b,
                         const double *F, const int64_t *f_offset,
                         const double *U_in, double *U_out)
{
    if (check_params(prm) != REF_OK || check_batch(b) != REF_OK) return REF_EINVAL;
    if (b->n_sub > 0 && (!F || !f_offset || !U_in || !U_out)) return REF_EINVAL;
    for (int s = 0; s < b->n_sub; s++)
        divergence_subgrid(F + f_offset[s], U_in + b->offset[s], U_out + b->offset[s],
                           b->fstride, 6 + b->n_species[s], prm->dt, b->h[s]);
    return REF_OK;
}

int hydro_ref_step(const hydro_ref_params *prm, const hydro_ref_batch *b,
                   const double *U_in, double *U_out, double *amax, int32_t *status)
{
    if (check_params(prm) != REF_OK || check_batch(b) != REF_OK) return REF_EINVAL;
    if (b->n_sub > 0 && (!U_in || !U_out || !amax)) return REF_EINVAL;
    double *Q = (double *)malloc(sizeof(double) * hydro_ref_q_elems(5));
    double *F = (double *)malloc(sizeof(double) * hydro_ref_f_elems(5));
    if (!Q || !F) { free(Q); free(F); return REF_EINVAL; }
    for (int s = 0; s < b->n_sub; s++) {
        int nf = 6 + b->n_species[s];
        const double *U = U_in + b->offset[s];
        reconstruct_subgrid(prm, U, b->fstride, nf, Q);
        double a;
        int bits = flux_subgrid(prm, Q, nf, F, &a);
        bits |= divergence_subgrid(F, U, U_out + b->offset[s], b->fstride, nf,
                                   prm->dt, b->h[s]);
        amax[s] = a;
        if (status) status[s] = bits;
    }
    free(Q);
    free(F);
    return REF_OK;
}

/* ---- entropy-tracer re-synchronisation (after a stage) ------------------------
 *
 * In a dual-energy scheme the entropy tracer tau stands in for the internal
 * energy only where e_i = E - |s|^2/(2 rho) is unreliable (e_i < eps E, the
 * same switch as in the point state); everywhere else tau is reset from the
 * total energy so that the two stay consistent: tau = e_i^(1/gamma).  Interior
 * cells only; U is updated in place.  Returns REF_OK or REF_EINVAL.
 */
int hydro_ref_tau_resync(const hydro_ref_params *prm, const hydro_ref_batch *b, double *U)
{
    if (check_params(prm) != REF_OK || check_batch(b) != REF_OK) return REF_EINVAL;
    if (b->n_sub > 0 && !U) return REF_EINVAL;
    for (int s = 0; s < b->n_sub; s++) {
        double *Us = U + b->offset[s];
        const int64_t fs = b->fstride;
        for (int k = IL; k < IH; k++)
            for (int j = IL; j < IH; j++)
                for (int i = IL; i < IH; i++) {
                    const int c = cell_index(i, j, k);
                    const double rho = Us[F_RHO * fs + c];
                    const double sx = Us[(F_SX + 0) * fs + c];
                    const double sy = Us[(F_SX + 1) * fs + c];
                    const double sz = Us[(F_SX + 2) * fs + c];
                    const double E = Us[F_EGAS * fs + c];
                    const double r = 1.0 / rho;
                    const double vx = sx * r, vy = sy * r, vz = sz * r;
                    const double ek = 0.5 * ((sx * vx + sy * vy) + sz * vz);
                    const double ei = E - ek;
                    if (!(ei < prm->de_switch * E))
                        Us[F_TAU * fs + c] = pow(ei, 1.0 / prm->gamma);
                }
    }
    return REF_OK;
}
