// fused.hip -- the fused hydro stage: PPM reconstruction, central-upwind
// flux with Simpson quadrature and the finite-volume update in one persistent
// launch, with no intermediate array in HBM.
//
// Mapping (one workgroup of 8 waves per subgrid, looping over subgrids):
//   * The subgrid is swept plane by plane along z.  LDS holds a rolling
//     window of 5 z-planes of every field (planes k-2..k+2 around the current
//     plane k); the next plane is prefetched into registers one step ahead.
//   * Four roles, each split over two waves by field group: the "hydro" wave
//     (density, momenta, energy, tau and the point states) and the "species"
//     wave (the passive scalars).  Roles 0, 1, 2 own the x-, y- and z-faces
//     of the 8x8 interior cells of plane k (lane = cell); the 13 PPM lines of
//     a cell are produced once each over 5 rounds, and every line's two
//     surface points go through LDS to each role whose faces contain them.
//     The rounds are scheduled so that no owner consumes more than two lines
//     per round.  Role 3 handles the 32 "ring" cells just outside the
//     interior in x and y (2 lanes each), which only need the 9 points of the
//     face they share with the interior.  The hydro and species waves of a
//     role sit on the same SIMD, which keeps two waves per SIMD.
//   * The flux of a face is linear in the Simpson-weighted point terms once
//     its speeds a+, a- are known, so each side accumulates
//         S_V = sum w V,  S_F = sum w F(V),  lambda+- = max/min u_n +- c
//     over its 9 points, and the face flux is formed once both sides are done:
//         F = (a+ S_F^L - a- S_F^R + a+ a- (S_V^R - S_V^L)) / (a+ - a-).
//   * z-faces are carried from one plane step to the next; a plane's cells
//     are updated one step after their x/y fluxes are known.
// All floating point is FP64 on the vector ALUs.
#include "hydro_internal.hpp"

namespace hydro {

static_assert(NSUB == 8, "the fused kernel maps the 8x8 cells of a plane onto a 64-lane wave");

namespace {

// Row pitch of the blocks in global memory (GNB) and the global offset,
// within a plane, of window cell c = j NB + i.  The LDS window always holds
// NB-double rows; a library that steps the 8^3 tiles of larger blocks in
// place (the 16^3 build) compiles this file with HYDRO_FUSED_GNB set to that
// block's edge.
#ifdef HYDRO_FUSED_GNB
constexpr int GNB = HYDRO_FUSED_GNB;
#define GCELL(c) (((c) / NB) * GNB + (c) % NB)
#else
constexpr int GNB = NB;
#define GCELL(c) (c)
#endif
constexpr int GNP = GNB * GNB;
static_assert(GNB >= NB, "a block row holds the tile's row");

constexpr int NT = 512;                 // 8 waves
constexpr int SLOTS = 5;                // window planes
constexpr int PT = 16;                  // doubles per exchanged point
constexpr int P_VX = 11, P_P = 14, P_CS = 15;   // point slots after V[0..10]
constexpr int NH = 14;                  // hydro partial: sv[0..5] sf[1..5] sp lp lm
constexpr int NACC = NH + 10;           // one face side in LDS (+ species sv, sf)
constexpr int H_SP = 11, H_LP = 12, H_LM = 13;

// LDS layout, in doubles
constexpr int SLOT_D = NF_MAX * NPLANE + 2;          // one window plane, + a dummy word
constexpr int WIN_D = SLOTS * SLOT_D;                // 10790
constexpr int XCH_D = 3 * 2 * PT * 64;               // 6144
constexpr int ZL_D = NACC * 64;                      // 1536
constexpr int KEEP_D = 2 * NF_MAX * 64;              // 1408
constexpr int RUN_D = 6 * 64;                        // ring lanes: u_n and 5 species
constexpr int LDS_D = WIN_D + XCH_D + ZL_D + KEEP_D + RUN_D + 16;
static_assert(LDS_D * 8 <= 163840, "LDS budget");

// combine-phase sub-regions of XCH.  The face fluxes lie in the slots of
// the z-line producer, which is idle in the first round: the x owner reads
// them to form its cells' flux differences while the next step's first
// round is already being produced, with no barrier in between.
constexpr int RST = 2 * 8 * 9;                       // stride of one component
constexpr int XR_OFF = 0;                            // [24][2][8][9] right partials
constexpr int LL_OFF = NACC * RST;                   // [2][2][8][9] left speeds
constexpr int ZB_OFF = LL_OFF + 2 * RST;             // [4][64] z-face speeds
constexpr int XF_OFF = 2 * 2 * PT * 64;              // [11][2][8][9] face fluxes
static_assert(ZB_OFF + 4 * 64 <= XF_OFF, "combine layout");
static_assert(XF_OFF >= 4 * PT * 64 && XF_OFF + NF_MAX * RST <= XCH_D,
              "the face fluxes must lie outside round 0's and the face layers' exchange slots");

// ---- the 13 lines: n = 14 + L, (dx,dy,dz) from the base-3 digits of n -------

__device__ __host__ constexpr int ldx(int L) { return (14 + L) % 3 - 1; }
__device__ __host__ constexpr int ldy(int L) { return ((14 + L) / 3) % 3 - 1; }
__device__ __host__ constexpr int ldz(int L) { return (14 + L) / 9 - 1; }

// Lines produced by role w in round r (-1: idle).  Each round's lines cross
// every axis at most twice, so no face owner consumes more than two lines per
// round: rounds 0-1 hold the four body diagonals, rounds 2-3 one face
// diagonal of each plane, round 4 the three axes.
__device__ __host__ constexpr int line_of(int w, int r) {
    return w == 0 ? (r == 0 ? 12 : r == 1 ? -1 : r == 2 ? 1 : r == 3 ? 3 : 0)
         : w == 1 ? (r == 0 ? 10 : r == 1 ? 6 : r == 2 ? 7 : r == 3 ? 9 : 2)
                  : (r == 0 ? -1 : r == 1 ? 4 : r == 2 ? 5 : r == 3 ? 11 : 8);
}

static_assert(line_of(2, 0) < 0, "the z-line producer must be idle in round 0 (see XF_OFF)");

__device__ __host__ constexpr int comp(int L, int axis) {
    return axis == 0 ? ldx(L) : axis == 1 ? ldy(L) : ldz(L);
}

// Producer of the j-th line that crosses the faces of axis ax in round r
// (round 4 has one such line; j = 1 repeats it).
__device__ __host__ constexpr int cons_producer(int ax, int r, int j) {
    return r == 4 ? ax
         : r == 1 ? 1 + j
         : r == 0 ? j
         : ax == 0 ? j
         : ax == 1 ? 2 * j
                   : 1 + j;
}

// The t-th line (t = 0..8) that crosses the z faces, in the order in which the
// z-face owner of an interior plane step sums them (rounds 0-4, two lines a
// round, one in the last).  The face layers sum their points in this order
// too, so a z face comes out bit for bit the same whether its sides were
// produced in interior steps or in face layers.
__device__ __host__ constexpr int zline(int t) {
    return line_of(cons_producer(2, t / 2, t % 2), t / 2);
}

__host__ constexpr bool zlines_ok() {
    for (int t = 0; t < 9; t++) {
        if (zline(t) < 0 || ldz(zline(t)) != 1) return false;
        for (int u = 0; u < t; u++)
            if (zline(u) == zline(t)) return false;
    }
    return true;
}
static_assert(zlines_ok(), "the nine z-crossing lines, each once");

// Line directions in 6 bits: dx + 1, dy + 1, dz + 1, two bits each.
__device__ __host__ constexpr int dir_code(int L) {
    return (ldx(L) + 1) | ((ldy(L) + 1) << 2) | ((ldz(L) + 1) << 4);
}

// The lines of role w (0-2) over the 5 rounds, 7 bits a round (bit 6: a line
// is produced; bits 0-5 its direction code), and the nine z lines of the face
// layers in the order zline, 6 bits each: uniform lookups by shifts, where the
// definitions above compile into chains of scalar branches.
__device__ __host__ constexpr uint64_t prod_table(int w) {
    uint64_t t = 0;
    for (int r = 0; r < 5; r++)
        if (line_of(w, r) >= 0) t |= (uint64_t)(64 | dir_code(line_of(w, r))) << (7 * r);
    return t;
}

__device__ __host__ constexpr uint64_t zline_dirs() {
    uint64_t t = 0;
    for (int u = 0; u < 9; u++) t |= (uint64_t)dir_code(zline(u)) << (6 * u);
    return t;
}

__host__ constexpr bool tables_ok() {
    for (int w = 0; w < 3; w++)
        for (int r = 0; r < 5; r++) {
            const int pd = (int)(prod_table(w) >> (7 * r)) & 127;
            const int L = line_of(w, r);
            if ((L >= 0) != ((pd & 64) != 0)) return false;
            if (L >= 0 && ((pd & 3) - 1 != ldx(L) || ((pd >> 2) & 3) - 1 != ldy(L) ||
                           ((pd >> 4) & 3) - 1 != ldz(L)))
                return false;
        }
    for (int u = 0; u < 9; u++) {
        const int dc = (int)(zline_dirs() >> (6 * u)) & 63;
        if ((dc & 3) - 1 != ldx(zline(u)) || ((dc >> 2) & 3) - 1 != ldy(zline(u)) ||
            (dc >> 4) - 1 != ldz(zline(u)))
            return false;
    }
    return true;
}
static_assert(tables_ok(), "packed line tables decode to the schedule");

// Simpson weight codes of the nine z lines (see simpson_wc), two bits each.
__device__ __host__ constexpr uint32_t zline_wcodes() {
    uint32_t t = 0;
    for (int u = 0; u < 9; u++)
        t |= (uint32_t)(1 + (ldx(zline(u)) == 0) + (ldy(zline(u)) == 0)) << (2 * u);
    return t;
}

// Simpson weight of a surface point from its two tangential offsets.
__device__ __forceinline__ double simpson_w(int t1, int t2) {
    const double w1a = t1 == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
    const double w1b = t2 == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
    return w1a * w1b;
}

// The same weights by code: 0 for none, else 1 + the number of zero offsets
// (the products are formed as in simpson_w, so the bits agree).
__device__ __forceinline__ double simpson_wc(int c) {
    constexpr double e = 1.0 / 6.0, m = 4.0 / 6.0;
    constexpr double w1 = e * e, w2 = m * e, w3 = m * m;
    return c == 0 ? 0.0 : c == 1 ? w1 : c == 2 ? w2 : w3;
}

// What the owner of the axis-ax faces takes from the j-th line it consumes in
// round r, in 5 bits: the exchange slot of the point on its cells' + side
// (the producer's + or - slot, by the sign of the line's ax component; the
// other side's point is in the slot next to it, slot ^ 1), and in bits 3-4
// the Simpson weight code (0 for the repeated line of the last round).
__device__ __host__ constexpr int cons_desc(int ax, int r, int j) {
    const int p = cons_producer(ax, r, j);
    const int Lp = line_of(p, r);
    const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
    const int slot = p * 2 + (comp(Lp, ax) > 0 ? 0 : 1);
    const int wc = (r == 4 && j == 1) ? 0 : 1 + (comp(Lp, b1) == 0) + (comp(Lp, b2) == 0);
    return slot | (wc << 3);
}

// The ten descriptors of axis ax, packed: the j-th line of round r at bit
// 5 (2 r + j).  Uniform lookups with shifts keep the consumption straight-line
// code, so all of a round's loads can be issued before the first sum.
__device__ __host__ constexpr uint64_t cons_table(int ax) {
    uint64_t t = 0;
    for (int r = 0; r < 5; r++)
        for (int j = 0; j < 2; j++) t |= (uint64_t)cons_desc(ax, r, j) << (5 * (2 * r + j));
    return t;
}

// Each entry of the consumption tables names a slot of a line that crosses
// the owner's faces and was produced in that round, on the owner's + side.
__host__ constexpr bool cons_tables_ok() {
    for (int ax = 0; ax < 3; ax++)
        for (int r = 0; r < 5; r++)
            for (int j = 0; j < 2; j++) {
                const int d = (int)(cons_table(ax) >> (5 * (2 * r + j))) & 31;
                const int p = (d & 7) >> 1, L = line_of(p, r);
                if (L < 0 || comp(L, ax) == 0 || (comp(L, ax) > 0) != ((d & 1) == 0)) return false;
                if ((d >> 3) == 0 && !(r == 4 && j == 1)) return false;
            }
    return true;
}
static_assert(cons_tables_ok(), "consumption tables");

// ---- PPM in branch-free form ---------------------------------------------

// Twice the monotonised-central slope from the two one-sided differences:
// sign(d) max(0, min(|dm + dp|, 4 min(sg dm, sg dp))), sg the sign of the
// centred difference d = (dm + dp) / 2.  Halving is exact unless dm + dp is
// subnormal, so this is bit for bit 2 x the slope min(|d|, 2|dm|, 2|dp|)
// (zero unless dm and dp share d's sign), with one multiplication fewer.  The sign is applied by
// multiplication (the values stay ordinary floats, so min/max need no NaN
// canonicalisation).
__device__ __forceinline__ double mc_slope2(double dm, double dp) {
    const double sum = dm + dp;
    const double sg = copysign(1.0, sum);
    const double t = fmin(dm * sg, dp * sg);    // > 0 only if both share d's sign
    return fmax(fmin(fabs(sum), 4.0 * t), 0.0) * sg;
}

// PPM on u_{-2..2}: the Colella-Woodward monotonicity step written in its
// equivalent clamp form (a = q+ - u0, b = u0 - q-: flatten if a b <= 0, else
// |b| <= 2|a| and |a| <= 2|b|), which needs no division and no branches.
__device__ __forceinline__ void ppm_fast(double um2, double um1, double u0, double up1,
                                         double up2, double &qp, double &qm) {
    // Twice the offsets: with the slopes doubled, 2 (q+ - u0) = d+ + (S0 - S+)/6
    // and 2 (u0 - q-) = d- + (S0 - S-)/6, each one rounding of an exact
    // multiple of the undoubled value, so every quantity below is an exact
    // power-of-two multiple of the undoubled form's and q+, q- are the same
    // bits (for differences above the subnormal range, where halving rounds).
    const double sixth = 1.0 / 6.0;
    double d0 = um1 - um2, d1 = u0 - um1, d2 = up1 - u0, d3 = up2 - up1;
    double sm = mc_slope2(d0, d1);
    double s0 = mc_slope2(d1, d2);
    double sp = mc_slope2(d2, d3);
    const double A = fma(s0 - sp, sixth, d2);   // 2 (q+ - u0)
    const double B = fma(s0 - sm, sixth, d1);   // 2 (u0 - q-)
    const double h = copysign(0.5, A);          // sign of a, halved
    const double sb = B * h;                    // |b| if b has a's sign, else < 0
    const double bn = fmax(fmin(sb, fabs(A)), 0.0);           // min(|b|, 2|a|), or 0
    const double An = fmax(fmin(fabs(A), 4.0 * sb), 0.0);     // 2 min(|a|, 2|b|), or 0
    qp = fma(An, h, u0);
    qm = fma(bn, -(h + h), u0);
}

// ppm_fast with the Colella-Woodward weights applied to the interface offsets
// before the monotonicity step: steepening (eta) moves q+ toward
// u_{+1} - s_{+1}/2 and q- toward u_{-1} + s_{-1}/2, flattening (flat) moves
// both toward u0.  With eta = flat = 0 it is ppm_fast.
__device__ __forceinline__ void ppm_fast_w(double um2, double um1, double u0, double up1,
                                           double up2, double eta, double flat, double &qp,
                                           double &qm) {
    const double twelfth = 1.0 / 12.0;
    double d0 = um1 - um2, d1 = u0 - um1, d2 = up1 - u0, d3 = up2 - up1;
    double sm = mc_slope2(d0, d1);                // doubled slopes, as in ppm_fast
    double s0 = mc_slope2(d1, d2);
    double sp = mc_slope2(d2, d3);
    double a = fma(s0 - sp, twelfth, 0.5 * d2);
    double b = fma(s0 - sm, twelfth, 0.5 * d1);
    a = fma(eta, fma(-0.25, sp, d2) - a, a);      // -s/2 = -S/4
    b = fma(eta, fma(-0.25, sm, d1) - b, b);
    const double keep = 1.0 - flat;
    a *= keep;
    b *= keep;
    double sg = copysign(1.0, a);
    double aa = fabs(a);
    double sb = b * sg;
    double bn = fmax(fmin(sb, aa + aa), 0.0);
    double an = fmax(fmin(aa, sb + sb), 0.0);
    qp = fma(an, sg, u0);
    qm = fma(-bn, sg, u0);
}

// 1/x from the hardware estimate and two Newton steps (each doubles the
// number of correct bits; the result is within an ulp of the rounded quotient).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Square root for the sound speed: Goldschmidt's iteration from the hardware
// reciprocal-square-root estimate (root g and half-reciprocal h refined
// together), then two Newton corrections of the root, g += (x - g^2) h.  This
// is the arithmetic of the device library's sqrt without its rescaling of
// arguments below 2^-767 (a squared sound speed is never that small); zero
// and infinity pass through, negative and NaN arguments give NaN.
__device__ __forceinline__ double sqrt_cs(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    d = fma(-g, g, x);
    g = fma(d, h, g);
    return (x == 0.0 || x == INFINITY) ? x : g;
}

// tau^gamma for the dual-energy branch.  For the paper's gas, gamma = 5/3,
// tau^(5/3) = tau * (tau * tau^(-1/3)) with y = tau^(-1/3) from Newton's
// iteration for the inverse cube root, y <- y (4 - x y^3) / 3 (quadratic
// convergence): the exponent is split off exactly (x = m 2^(3q)), a
// single-precision estimate of m^(-1/3) (about 22 correct bits) is refined
// twice in double precision.  The result is within 4 ulp of x^(5/3); it
// differs from pow(x, 5/3 rounded to double) by the rounding of the
// exponent, a relative 4e-17 |ln x|.  Other gamma, and tau that is not a
// positive finite number, take the library pow.
__device__ __forceinline__ double tau_pow(double x, double gamma) {
    if (gamma == 5.0 / 3.0 && x > 0.0 && x < INFINITY) {
        int e = __builtin_amdgcn_frexp_exp(x);        // x = m 2^e, m in [0.5, 1)
        double m = __builtin_amdgcn_frexp_mant(x);
        int q = (e >= 0 ? e : e - 2) / 3;              // floor(e / 3)
        m = __builtin_amdgcn_ldexp(m, e - 3 * q);      // m in [0.5, 4)
        const float mf = (float)m;
        double y = (double)__builtin_amdgcn_exp2f(-0.333333333f * __builtin_amdgcn_logf(mf));
        const double third = 1.0 / 3.0;
#pragma unroll
        for (int it = 0; it < 2; it++) {
            const double y3 = (y * y) * y;
            y = (y * third) * fma(-m, y3, 4.0);
        }
        y = __builtin_amdgcn_ldexp(y, -q);             // x^(-1/3)
        return x * (x * y);
    }
    return pow(x, gamma);
}

// The value of lane ^ 1 (the other lane of a pair), by a DPP quad
// permutation [1, 0, 3, 2] of both halves: no LDS round trip.
__device__ __forceinline__ double pair_swap(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS accesses,
// not for its global loads and stores (which never carry data between waves).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Hide a value from loop-invariant code motion: address arithmetic derived
// from it is recomputed where it is used instead of being hoisted out of the
// plane loop and kept live (which would exhaust the register file).
// Compile-time scheduling fence: keeps the scheduler from hoisting the loads
// of one stage above the previous one (which would raise register pressure).
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

template <typename T>
__device__ __forceinline__ T opaque_s(T v) {
    asm volatile("" : "+s"(v));
    return v;
}
template <typename T>
__device__ __forceinline__ T opaque_v(T v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Per-lane geometry, re-derived from an opaque thread index at the top of each
// phase so that none of it is hoisted out of the loops and kept live:
// (ci, cj) is the lane's interior cell of the plane; role-3 lanes own ring
// cell rc = lane/2 (x-ring for rc < 16, else y-ring; low or high side).
#define LANE_GEOMETRY()                                                          \
    const int lane = opaque_v((int)threadIdx.x) & 63;                            \
    const int ci = 3 + (lane & 7), cj = 3 + ((((lane >> 3) & 1) << 2) | (lane >> 4)); \
    const int half = lane & 1;                                                   \
    const int r_axis = (lane >> 1) >> 4, r_side = ((lane >> 1) >> 3) & 1;        \
    const int r_pos = 3 + ((lane >> 1) & 7);                                     \
    const int ri = r_axis == 0 ? (r_side ? 11 : 2) : r_pos;                      \
    const int rj = r_axis == 0 ? r_pos : (r_side ? 11 : 2);                      \
    (void)ci; (void)cj; (void)half; (void)r_axis; (void)r_side; (void)r_pos;     \
    (void)ri; (void)rj

// ---- ghost cells read through a ghost map -------------------------------------

// Source of a block cell of plane pk when the ghost layers are read through a
// ghost map (the ghost fill's rule, applied on load).  The cell is packed in g:
// bits 0-3 i, 4-7 j, 8-9 dx + 1, 10-11 dy + 1 (its ghost direction in x and
// y); fo is its field's offset.  The direction picks the table entry (entry
// 13, the interior, is the subgrid itself); along each axis the index steps
// N cells back into the neighbour, or clamps to the nearest interior cell
// where the entry's mode bit for that axis is set.
__device__ __forceinline__ const double *gather_ptr(const double *U, const int64_t *toff,
                                                    const int *tmode, int fo, int g, int pk) {
    const int i = g & 15, j = (g >> 4) & 15;
    const int dx = ((g >> 8) & 3) - 1, dy = ((g >> 10) & 3) - 1;
    const int dz = pk < NG ? -1 : (pk >= NG + NSUB ? 1 : 0);
    const int n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
    const int m = tmode[n];
    const int si = dx == 0 ? i : ((m & 1) ? (dx < 0 ? NG : NG + NSUB - 1) : i - NSUB * dx);
    const int sj = dy == 0 ? j : ((m & 2) ? (dy < 0 ? NG : NG + NSUB - 1) : j - NSUB * dy);
    const int sk = dz == 0 ? pk : ((m & 4) ? (dz < 0 ? NG : NG + NSUB - 1) : pk - NSUB * dz);
    return U + toff[n] + fo + (sk * NB + sj) * NB + si;
}

// ---- LDS window access --------------------------------------------------------

// The five window offsets of the line through (i,j,k) along (dx,dy,dz).
struct Line5 {
    int o[5];
};

__device__ __forceinline__ Line5 line5(int i, int j, int k, int dx, int dy, int dz) {
    Line5 l;
#pragma unroll
    for (int m = -2; m <= 2; m++) {
        int pl = (k + m * dz) % SLOTS;
        l.o[m + 2] = pl * SLOT_D + (j + m * dy) * NB + (i + m * dx);
    }
    return l;
}

// ---- Colella-Woodward steepening and flattening (the CW instantiation) ------

// Weights of one line: eta (contact steepening, density only) and flat
// (flattening, every field).
struct CwW {
    double eta, flat;
};

// Pressure and velocity along (dx, dy, dz) of the window cell at offset o,
// with the point-state formulas (dual-energy switch included).  The
// detectors that take these are discontinuous in them, and a cell's weights
// are formed again by every wave whose lines pass through it -- at a
// subgrid's edge by both neighbours, which must agree for the face flux to
// be conservative -- so the arithmetic is fixed: no contraction and the
// rounded quotient (the dual-energy branch takes tau_pow, as the point
// states do).  Without VEL it is the definition's order: v = s (1/rho),
// e_k = (s.v)/2.  With VEL the momentum slots hold the correctly rounded
// quotients s / rho, which are taken as v, and e_k = ((rho v).v)/2; these
// differ from the definition's values in the last bits, so near a
// detector's threshold a weight can differ from the definition's (parity
// for this combination is checked on inputs whose detectors sit away from
// their thresholds).
template <bool VEL>
__device__ __forceinline__ void cw_cell(const double *win, int o, int dx, int dy, int dz,
                                        double gamma, double gm1, double de, double &p,
                                        double &un) {
#pragma clang fp contract(off)
    const double rho = win[o];
    const double m1 = win[o + NPLANE], m2 = win[o + 2 * NPLANE], m3 = win[o + 3 * NPLANE];
    double vx, vy, vz, ek;
    if (VEL) {
        vx = m1;
        vy = m2;
        vz = m3;
        ek = 0.5 * (((rho * vx) * vx + (rho * vy) * vy) + (rho * vz) * vz);
    } else {
        const double r = 1.0 / rho;
        vx = m1 * r;
        vy = m2 * r;
        vz = m3 * r;
        ek = 0.5 * ((m1 * vx + m2 * vy) + m3 * vz);
    }
    const double E = win[o + 4 * NPLANE];
    double ei = E - ek;
    if (ei < de * E) ei = tau_pow(win[o + 5 * NPLANE], gamma);
    p = gm1 * ei;
    un = (dx * vx + dy * vy) + dz * vz;
}

// The weights of the line l along (dx, dy, dz).  mode: bit 0 steepening, bit 1
// flattening.  Flattening: in a compression along the line with a relative
// pressure jump above eps, clamp(omega2 ((p_1 - p_-1) / (p_2 - p_-2) -
// omega1), 0, 1), the ratio +inf where p_2 = p_-2.  Steepening: where the density's second differences on the
// two sides have opposite signs, its jump exceeds eps1 of the smaller density
// and gamma K0 |jump| / min rho >= |p_1 - p_-1| / min p, clamp(eta1 (eta~ -
// eta2), 0, 1) with eta~ = -(D_1 - D_-1) / (6 (rho_1 - rho_-1)).  Both are
// taken with selects (the lanes differ).
template <bool VEL>
__device__ __forceinline__ CwW cw_weights(const double *win, const Line5 &l, int dx, int dy,
                                          int dz, double gamma, double gm1, double de, int mode,
                                          bool need_eta) {
#pragma clang fp contract(off)
    double p[5], un[5];
#pragma unroll
    for (int m = 0; m < 5; m++)
        if (m != 2) cw_cell<VEL>(win, l.o[m], dx, dy, dz, gamma, gm1, de, p[m], un[m]);
    CwW w;
    w.eta = 0.0;
    w.flat = 0.0;
    if (mode & 2) {
        const double dp1 = p[3] - p[1];
        const bool shock = (un[1] - un[3] > 0.0) && (fabs(dp1) / fmin(p[3], p[1]) > CW_EPS_SHOCK);
        const double dp2 = p[4] - p[0];
        // equal outer pressures: +inf in either direction of the line
        const double ratio = dp2 != 0.0 ? dp1 / dp2 : INFINITY;
        const double f = fmax(0.0, fmin(1.0, CW_OMEGA2 * (ratio - CW_OMEGA1)));
        w.flat = shock ? f : 0.0;
    }
    if ((mode & 1) && need_eta) {
        double r[5];
#pragma unroll
        for (int m = 0; m < 5; m++) r[m] = win[l.o[m]];
        // outer pair first: a line and its reverse give the same bits
        const double d2m = (r[0] + r[2]) - 2.0 * r[1];
        const double d2p = (r[2] + r[4]) - 2.0 * r[3];
        const double drho = r[3] - r[1];
        const bool contact =
            (d2p * d2m < 0.0) &&
            (fabs(drho) - CW_EPS1 * fmin(fabs(r[3]), fabs(r[1])) > 0.0) &&
            (gamma * CW_K0 * fabs(drho) / fmin(r[3], r[1]) >= fabs(p[3] - p[1]) / fmin(p[3], p[1]));
        const double et = -(d2p - d2m) / (6.0 * drho);
        const double e = fmax(0.0, fmin(CW_ETA1 * (et - CW_ETA2), 1.0));
        w.eta = contact ? e : 0.0;
    }
    return w;
}

// The five window values of field f along l.
struct Pts5 {
    double u[5];
};

__device__ __forceinline__ Pts5 load5(const double *win, const Line5 &l, int f) {
    const int fo = f * NPLANE;
    Pts5 p;
#pragma unroll
    for (int m = 0; m < 5; m++) p.u[m] = win[l.o[m] + fo];
    return p;
}

// PPM of field f from its five values: plain, or with the line's weights
// (eta for the density only).
template <bool CW>
__device__ __forceinline__ void ppm_pts(const Pts5 &p, int f, const CwW &w, double &qp,
                                        double &qm) {
    if (!CW) ppm_fast(p.u[0], p.u[1], p.u[2], p.u[3], p.u[4], qp, qm);
    else ppm_fast_w(p.u[0], p.u[1], p.u[2], p.u[3], p.u[4], f == 0 ? w.eta : 0.0, w.flat, qp, qm);
}

// PPM of fields F0..F1-1 along l, handing each field's values to sink(f, q+,
// q-).  A field's loads are issued before the previous field is
// reconstructed: the sinks store to LDS, which the compiler cannot tell apart
// from the window, so loads placed after a store would wait for it and leave
// the load latency exposed field by field.
template <bool CW, int F0, int F1, typename Sink>
__device__ __forceinline__ void ppm_fields(const double *win, const Line5 &l, const CwW &cw,
                                           Sink &&sink) {
    Pts5 c = load5(win, l, F0);
#pragma unroll
    for (int f = F0; f < F1; f++) {
        Pts5 n = c;
        if (f + 1 < F1) n = load5(win, l, f + 1);
        sched_fence();   // keep the loads ahead of the reconstruction
        double qp, qm;
        ppm_pts<CW>(c, f, cw, qp, qm);
        sink(f, qp, qm);
        c = n;
    }
}

// ---- producers ------------------------------------------------------------------

// Hydro fields along one line: reconstructed values and the point states at
// both ends, written to the exchange slots as they are formed (component
// stride 64) when `store`; with `both` false only the + point is formed, and
// with `minus_only` only the - point (stored at pm).
// With VEL the window holds the velocities s / rho in the momentum slots:
// their PPM values are the point velocities, and the point momenta are those
// times the point density.
struct PlusState {
    double q[6];
    double vx, vy, p, cs;
};

// The loads of field f + 1 are issued before field f is reconstructed (see
// ppm_fields); with XF >= 0 the values of field XF are loaded the same way
// during the last hydro field and returned in xv.  VXO is the slot of the
// stored point's x velocity (then y, z, pressure and sound speed follow):
// P_VX for the 16-double point of the 11-field plan, 6 for the 11-double
// point of the plane-paired plan.
template <bool store_, bool both_, bool VEL, bool CW, bool minus_only = false, int XF = -1,
          int VXO = P_VX>
__device__ __forceinline__ PlusState produce_hydro(const double *win, const Line5 &l,
                                                   double *pp, double *pm, double gamma,
                                                   double gm1, double de, int &bits,
                                                   const CwW &cw, Pts5 *xv = nullptr) {
    constexpr bool plus = !minus_only, store = store_ && plus, both = both_ || minus_only;
    PlusState ps;
    double qp, qm;
    Pts5 c = load5(win, l, 0), n = load5(win, l, 1);
    sched_fence();
    ppm_pts<CW>(c, 0, cw, qp, qm);
    ps.q[0] = qp;
    if (store) pp[0] = qp;
    if (both) pm[0] = qm;
    const double rhop = qp, rhom = qm;
    const double rp = plus ? recip(qp) : 1.0, rm = both ? recip(qm) : 1.0;
    c = load5(win, l, 2);
    sched_fence();
    ppm_pts<CW>(n, 1, cw, qp, qm);
    const double wxp = qp, wxm = qm;
    if (VEL) {
        qp = rhop * wxp;
        qm = rhom * wxm;
    }
    ps.q[1] = qp;
    if (store) pp[64] = qp;
    if (both) pm[64] = qm;
    const double vxp = VEL ? wxp : qp * rp, vxm = VEL ? wxm : qm * rm;
    double ekp = qp * vxp, ekm = qm * vxm;
    n = load5(win, l, 3);
    sched_fence();
    ppm_pts<CW>(c, 2, cw, qp, qm);
    const double wyp = qp, wym = qm;
    if (VEL) {
        qp = rhop * wyp;
        qm = rhom * wym;
    }
    ps.q[2] = qp;
    if (store) pp[2 * 64] = qp;
    if (both) pm[2 * 64] = qm;
    const double vyp = VEL ? wyp : qp * rp, vym = VEL ? wym : qm * rm;
    ekp = fma(qp, vyp, ekp);
    ekm = fma(qm, vym, ekm);
    c = load5(win, l, 4);
    sched_fence();
    ppm_pts<CW>(n, 3, cw, qp, qm);
    const double wzp = qp, wzm = qm;
    if (VEL) {
        qp = rhop * wzp;
        qm = rhom * wzm;
    }
    ps.q[3] = qp;
    if (store) pp[3 * 64] = qp;
    if (both) pm[3 * 64] = qm;
    const double vzp = VEL ? wzp : qp * rp, vzm = VEL ? wzm : qm * rm;
    ekp = fma(qp, vzp, ekp);
    ekm = fma(qm, vzm, ekm);
    n = load5(win, l, 5);
    sched_fence();
    ppm_pts<CW>(c, 4, cw, qp, qm);
    ps.q[4] = qp;
    if (store) pp[4 * 64] = qp;
    if (both) pm[4 * 64] = qm;
    const double Ep = qp, Em = qm;
    if (XF >= 0) *xv = load5(win, l, XF);
    sched_fence();
    ppm_pts<CW>(n, 5, cw, qp, qm);
    ps.q[5] = qp;
    if (store) pp[5 * 64] = qp;
    if (both) pm[5 * 64] = qm;
    double prp = 0.0, csp = 0.0;
    if (plus) {
        double eip = fma(-0.5, ekp, Ep);
        if (eip < de * Ep) eip = tau_pow(qp, gamma);      // dual energy: tau^gamma
        prp = gm1 * eip;
        csp = sqrt_cs((gamma * prp) * rp);
        if (store) {
            pp[VXO * 64] = vxp;
            pp[(VXO + 1) * 64] = vyp;
            pp[(VXO + 2) * 64] = vzp;
            pp[(VXO + 3) * 64] = prp;
            pp[(VXO + 4) * 64] = csp;
        }
        bits |= (__ballot(rhop <= 0.0) ? HYDRO_STATUS_RHO : 0) |
                (__ballot(prp <= 0.0) ? HYDRO_STATUS_P : 0);
    }
    if (both) {
        double eim = fma(-0.5, ekm, Em);
        if (eim < de * Em) eim = tau_pow(qm, gamma);
        const double prm = gm1 * eim;
        pm[VXO * 64] = vxm;
        pm[(VXO + 1) * 64] = vym;
        pm[(VXO + 2) * 64] = vzm;
        pm[(VXO + 3) * 64] = prm;
        pm[(VXO + 4) * 64] = sqrt_cs((gamma * prm) * rm);
        bits |= (__ballot(rhom <= 0.0) ? HYDRO_STATUS_RHO : 0) |
                (__ballot(prm <= 0.0) ? HYDRO_STATUS_P : 0);
    }
    ps.vx = vxp;
    ps.vy = vyp;
    ps.p = prp;
    ps.cs = csp;
    return ps;
}

// ---- accumulation of one surface point into a face-side partial ----------------
// Hydro waves use all NH slots; species waves use slots 0..4 (sv) and 5..9 (sf).

__device__ __forceinline__ void acc_zero(double (&c)[NH], bool hydro) {
#pragma unroll
    for (int i = 0; i < NH; i++) c[i] = 0.0;
    if (hydro) {
        c[H_LP] = -INFINITY;
        c[H_LM] = INFINITY;
    }
}

// a + b and a - b as single roundings, never fused with a product that forms
// a or b: a point's terms are formed in registers by the wave that produced
// it and read from LDS by the others, and every wave must round them alike
__device__ __forceinline__ double add_r(double a, double b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ double sub_r(double a, double b) {
#pragma clang fp contract(off)
    return a - b;
}

__device__ __forceinline__ void acc_h_vals(double (&c)[NH], const double *V, double un,
                                           double p, double cs, double w) {
    const double wun = w * un;
#pragma unroll
    for (int f = 0; f < 6; f++) c[f] = fma(w, V[f], c[f]);
    c[6] = fma(wun, V[1], c[6]);
    c[7] = fma(wun, V[2], c[7]);
    c[8] = fma(wun, V[3], c[8]);
    c[9] = fma(wun, add_r(V[4], p), c[9]);
    c[10] = fma(wun, V[5], c[10]);
    c[H_SP] = fma(w, p, c[H_SP]);
    c[H_LP] = fmax(c[H_LP], add_r(un, cs));
    c[H_LM] = fmin(c[H_LM], sub_r(un, cs));
}

// a point's hydro values (and normal velocity, pressure and sound speed),
// loaded ahead of their sums
struct HPt {
    double V[6], un, p, cs;
};

template <int VXO = P_VX>
__device__ __forceinline__ HPt load_h(const double *pt, int ax) {
    HPt h;
#pragma unroll
    for (int f = 0; f < 6; f++) h.V[f] = pt[f * 64];
    h.un = pt[(VXO + ax) * 64];
    h.p = pt[(VXO + 3) * 64];
    h.cs = pt[(VXO + 4) * 64];
    return h;
}

// a point's normal velocity and species values (always all 5 species slots:
// slots past the subgrid's species count hold values that are never stored,
// so no per-field branch splits the loads)
struct SPt {
    double un, v[5];
};

__device__ __forceinline__ SPt load_s(const double *pt, int ax) {
    SPt q;
    q.un = pt[(P_VX + ax) * 64];
#pragma unroll
    for (int i = 0; i < 5; i++) q.v[i] = pt[(6 + i) * 64];
    return q;
}

__device__ __forceinline__ void acc_s_pt(double (&c)[NH], const SPt &q, double w) {
    const double wun = w * q.un;
#pragma unroll
    for (int i = 0; i < 5; i++) {
        c[i] = fma(w, q.v[i], c[i]);
        c[5 + i] = fma(wun, q.v[i], c[5 + i]);
    }
}

// ---- partials in LDS (component stride st; hydro comps, then species) ----------

__device__ __forceinline__ void store_h(double *base, int st, const double (&c)[NH]) {
#pragma unroll
    for (int i = 0; i < NH; i++) base[i * st] = c[i];
}

// All five species slots, whatever the subgrid's species count: LDS work on
// species is never split by a branch on that count (each branch would end
// a run of loads and leave their latency exposed); the slots past the count
// carry values that no output takes.
__device__ __forceinline__ void store_s(double *base, int st, const double (&c)[NH]) {
#pragma unroll
    for (int i = 0; i < 5; i++) {
        base[(NH + i) * st] = c[i];
        base[(NH + 5 + i) * st] = c[5 + i];
    }
}

struct Speeds {
    double ap, am, inv, apam, amax_face;
};

__device__ __forceinline__ Speeds face_speeds(double lpL, double lmL, double lpR, double lmR,
                                              bool sym) {
    Speeds s;
    s.ap = fmax(0.0, fmax(lpL, lpR));
    s.am = fmin(0.0, fmin(lmL, lmR));
    if (sym) {   // one speed for both directions
        const double a = fmax(s.ap, -s.am);
        s.ap = a;
        s.am = -a;
    }
    s.inv = 1.0 / (s.ap - s.am);
    s.apam = s.ap * s.am;
    s.amax_face = fmax(s.ap, -s.am);
    return s;
}

// Hydro fluxes of a face from my partial (registers) and the other side's
// (LDS at o, stride st).  Writes Fb[0..5].
__device__ __forceinline__ Speeds combine_h(const double (&m)[NH], const double *o, int st,
                                            bool mine_left, int axis, bool sym, double *Fb) {
    const double mlp = m[H_LP], mlm = m[H_LM], olp = o[H_LP * st], olm = o[H_LM * st];
    const Speeds s = mine_left ? face_speeds(mlp, mlm, olp, olm, sym)
                               : face_speeds(olp, olm, mlp, mlm, sym);
    const double cm = mine_left ? s.ap : -s.am;     // coefficient of my S_F
    const double co = mine_left ? -s.am : s.ap;     // coefficient of the other S_F
    const double sg = mine_left ? 1.0 : -1.0;       // S_V^R - S_V^L = sg (other - mine)
    // density flux: S_V of the normal momentum (value selects, no indexing)
    const double m1 = m[1], m2 = m[2], m3 = m[3];
    const double ms = axis == 0 ? m1 : (axis == 1 ? m2 : m3);
    const double os = o[(1 + axis) * st];
    {
        const double X = fma(cm, ms, co * os), Y = s.apam * (sg * (o[0] - m[0]));
        Fb[0] = fma(Y, s.inv, X * s.inv);
    }
    const double msp = m[H_SP], osp = o[H_SP * st];
#pragma unroll
    for (int f = 1; f < 6; f++) {
        double sfm = m[5 + f], sfo = o[(5 + f) * st];
        if (f == 1 + axis) {
            sfm += msp;
            sfo += osp;
        }
        const double X = fma(cm, sfm, co * sfo), Y = s.apam * (sg * (o[f * st] - m[f]));
        Fb[f] = fma(Y, s.inv, X * s.inv);
    }
    return s;
}

// Species fluxes of a face, speeds given; the other side's species partial at o
// (all five slots, see store_s).
__device__ __forceinline__ void combine_s(const double (&m)[NH], const double *o, int st,
                                          bool mine_left, const Speeds &s, double *Fb) {
    const double cm = mine_left ? s.ap : -s.am;
    const double co = mine_left ? -s.am : s.ap;
    const double sg = mine_left ? 1.0 : -1.0;
#pragma unroll
    for (int i = 0; i < 5; i++) {
        const double sfm = m[5 + i], sfo = o[(NH + 5 + i) * st];
        const double dv = sg * (o[(NH + i) * st] - m[i]);
        Fb[6 + i] = fma(cm, sfm, co * sfo) * s.inv + (s.apam * dv) * s.inv;
    }
}

// Update of one interior cell of plane `kc` from its z flux Fz and the kept
// x/y difference: U_out = U - lam ((dFx + dFy) + dFz) for fields [f0, f1),
// or, for the rate form, U_out = -lam ((dFx + dFy) + dFz) with lam = 1/h.
// Runge-Kutta stage combination of the update (U0 of this subgrid, or null).
struct Stage {
    const double *U0;
    double c0, c1;
    bool identity;   // dt == 0: the stage returns U0
};

// chk collects 0 * v over the outputs: it stays 0 unless some v is not finite.
// With VEL the momenta are read from the input (the window holds velocities).
// The LDS reads and the arithmetic run over the field group's whole range
// ([0, 6) or [6, 11), fixed at compile time once f0 is), so they form one
// run of loads; only global memory is limited to the subgrid's fields.
template <bool VEL>
__device__ __forceinline__ void update_cell(const double *win, const double *keep, int lane,
                                            int kc, int ci, int cj, int f0, int f1,
                                            const double *Fz, double lam, bool rate,
                                            const Stage &stg, const double *Us, double *Os,
                                            int fst, double &chk) {
    const int cidx = opaque_v(kc * GNP + cj * GNB + ci);
    const int fs = opaque_s(fst);
    const int f1x = f0 == 0 ? 6 : NF_MAX;
    double vv[NF_MAX];
#pragma unroll
    for (int f = 0; f < NF_MAX; f++)
        if (f >= f0 && f < f1x) {
            const double dfz = Fz[f] - keep[f * 64 + lane];
            const double sxy = keep[(NF_MAX + f) * 64 + lane];
            const double u = (VEL && f >= 1 && f <= 3)
                                 ? Us[f * fs + cidx]
                                 : win[(kc % SLOTS) * SLOT_D + f * NPLANE + cj * NB + ci];
            vv[f] = (rate ? 0.0 : u) - lam * (sxy + dfz);
        }
#pragma unroll
    for (int f = 0; f < NF_MAX; f++)
        if (f >= f0 && f < f1x && f < f1) {
            double v = vv[f];
            if (stg.U0) {
                const double u0 = stg.U0[f * fs + cidx];
                v = stg.identity ? u0 : fma(stg.c0, u0, stg.c1 * v);
            }
            chk = fma(v, 0.0, chk);
            Os[f * fs + cidx] = v;
        }
}

// update_cell with the summed flux difference of each field given,
// dsum[f] = (dFx + dFy) + dFz: the z owner forms it before the second flux
// phase's barrier (it reads the kept values another wave overwrites after
// that barrier) and writes the cells after it, while the first round of the
// next step is produced.
template <bool VEL>
__device__ __forceinline__ void update_cell_sum(const double *win, int kc, int ci, int cj,
                                                int f0, int f1, const double *dsum, double lam,
                                                bool rate, const Stage &stg, const double *Us,
                                                double *Os, int fst, double &chk) {
    const int cidx = opaque_v(kc * GNP + cj * GNB + ci);
    const int fs = opaque_s(fst);
    const int f1x = f0 == 0 ? 6 : NF_MAX;
    double vv[NF_MAX];
#pragma unroll
    for (int f = 0; f < NF_MAX; f++)
        if (f >= f0 && f < f1x) {
            const double u = (VEL && f >= 1 && f <= 3)
                                 ? Us[f * fs + cidx]
                                 : win[(kc % SLOTS) * SLOT_D + f * NPLANE + cj * NB + ci];
            vv[f] = (rate ? 0.0 : u) - lam * dsum[f];
        }
#pragma unroll
    for (int f = 0; f < NF_MAX; f++)
        if (f >= f0 && f < f1x && f < f1) {
            double v = vv[f];
            if (stg.U0) {
                const double u0 = stg.U0[f * fs + cidx];
                v = stg.identity ? u0 : fma(stg.c0, u0, stg.c1 * v);
            }
            chk = fma(v, 0.0, chk);
            Os[f * fs + cidx] = v;
        }
}

// The work of one subgrid for one field group (HYD: hydro fields and point
// states; else: species).  Both instantiations execute the same sequence of
// barriers, so the hydro and species waves of a workgroup stay in step.
template <bool HYD, bool VEL, bool CW, bool GATHER>
__device__ __forceinline__ void subgrid_body(double *win, double *xch, double *zl, double *keep,
                                             double *run, int tid, int role, int nspec,
                                             const double *Us0, double *Os0, int fst0,
                                             double lam, bool rate, const Stage &stg, bool sym,
                                             int cwmode, double gamma, double gm1, double de,
                                             double &amax_l, int &bits, const FusedArgs &a, int s,
                                             const double *Ug, int64_t *toff, int *tmode, int kb,
                                             int ke) {
    const int nf = 6 + nspec;
    double chk = 0.0;
    const int f0 = HYD ? 0 : 6, f1 = HYD ? 6 : nf;     // this wave's fields
    constexpr int f1x = HYD ? 6 : NF_MAX;              // ... and its LDS range (see store_s)
    const bool work = HYD || nspec > 0;                 // a species wave without species idles
    // this thread's share of a plane: up to 5 of the nf*196 values.  Lanes
    // without an element load a valid address and store into the slot's
    // dummy word, so the loads carry no branches and issue back to back.
    int g_off[5], l_off[5];
    // With VEL a momentum element is stored as s / rho: its thread also loads
    // the density of the same cell.  Momenta are elements [NPLANE, 4 NPLANE),
    // which only the first two of a thread's five elements can be.
    static_assert(4 * NPLANE <= 2 * NT, "momentum elements must be among q = 0, 1");
    int r_off[2];
    bool mom[2];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const int e = tid + q * NT;
        const int f = e / NPLANE, c = e - f * NPLANE;
        const bool ok = e < nf * NPLANE;
        if (!GATHER) {
            g_off[q] = ok ? f * fst0 + GCELL(c) : 0;
        } else {
            // the element's block cell, its ghost direction in x and y, and
            // its field, packed (lanes without an element: an interior cell
            // of field 0)
            const int i = ok ? c % NB : NG, j = ok ? c / NB : NG;
            const int dx = i < NG ? -1 : (i >= NG + NSUB ? 1 : 0);
            const int dy = j < NG ? -1 : (j >= NG + NSUB ? 1 : 0);
            g_off[q] = i | (j << 4) | ((dx + 1) << 8) | ((dy + 1) << 10) | ((ok ? f : 0) << 12);
        }
        l_off[q] = ok ? f * NPLANE + c : NF_MAX * NPLANE;
        if (q < 2) {
            mom[q] = VEL && ok && f >= 1 && f <= 3;
            r_off[q] = GCELL(c);
        }
    }
    // source of element q of plane pk, and of the density of the same cell.
    // With GATHER the source is found through the map from the packed
    // geometry (the plane's z direction is the same for the whole wave).
    auto gsrc_of = [&](int q, int pk, bool field) -> const double * {
        const int g = opaque_v(g_off[q]);   // derived values are not hoisted and kept live
        return gather_ptr(Ug, toff, tmode, field ? (g >> 12) * fst0 : 0, g, pk);
    };
    auto src = [&](int q, int pk) -> const double * {
        if (!GATHER) return Us0 + (g_off[q] + pk * GNP);   // one 64-bit add, as an index
        return gsrc_of(q, pk, true);
    };
    auto src_rho = [&](int q, int pk) -> const double * {
        if (!GATHER) return Us0 + (r_off[q] + pk * GNP);
        return gsrc_of(q, pk, false);
    };

    lds_barrier();   // the previous subgrid's LDS reads are done
    if (GATHER) {
        // the ghost map's 27 entries, checked: a source must be a valid
        // subgrid with at least this subgrid's fields; otherwise (and for the
        // interior, entry 13) the subgrid itself with every axis clamped
        if (tid < 27) {
            const int64_t own = Us0 - Ug;
            int64_t o = own;
            int m = tid == 13 ? 0 : 7;
            if (tid != 13) {
                const int sb = a.gsrc[s * 27 + tid];
                bool good = sb >= 0 && sb < a.n_sub;
                if (good) {
                    const int ns2 = a.n_species[sb];
                    const int64_t o2 = a.offset[sb];
                    good = ns2 >= 0 && ns2 <= 5 && ns2 >= nspec && o2 >= 0 && !(o2 & 1);
                    if (good) {
                        o = o2;
                        m = a.gmode[s * 27 + tid];
                    }
                }
                if (!good) bits |= HYDRO_STATUS_BADMETA;
            }
            toff[tid] = o;
            tmode[tid] = m;
        }
        lds_barrier();
    }
    // window: planes kb-2..kb+2, then prefetch plane kb+3
    {
        double v[SLOTS][5];
#pragma unroll
        for (int pl = 0; pl < SLOTS; pl++)
#pragma unroll
            for (int q = 0; q < 5; q++) v[pl][q] = *src(q, kb - 2 + pl);
        if (VEL) {
#pragma unroll
            for (int pl = 0; pl < SLOTS; pl++)
#pragma unroll
                for (int q = 0; q < 2; q++) {
                    const double rho = *src_rho(q, kb - 2 + pl);
                    if (mom[q]) v[pl][q] = v[pl][q] / rho;
                }
        }
#pragma unroll
        for (int pl = 0; pl < SLOTS; pl++) {
            double *dst = win + ((kb - 2 + pl) % SLOTS) * SLOT_D;
#pragma unroll
            for (int q = 0; q < 5; q++) dst[l_off[q]] = v[pl][q];
        }
    }
    double pf[5], pr[2];
#pragma unroll
    for (int q = 0; q < 5; q++) pf[q] = *src(q, kb + 3);
    if (VEL) {
#pragma unroll
        for (int q = 0; q < 2; q++) pr[q] = *src_rho(q, kb + 3);
    }
    lds_barrier();

    double acc[2][NH];       // [0]: face + (or the ring / layer face), [1]: face -
    double Fb[NF_MAX];
    double dsum[NF_MAX];     // the z owner's summed flux differences of plane k-1
    for (int k = kb; k <= ke; k++) {
        const double *Us = Us0;
        double *Os = Os0;
        const int fst = opaque_s(fst0);
        (void)fst;
        acc_zero(acc[0], HYD);
        acc_zero(acc[1], HYD);

        // ---- rounds of line production and consumption.  Face layers (the
        // planes kb and ke just below and above the part's interior planes):
        // 3 rounds, every role produces one of the 9 points of the z face the
        // plane shares with the part (its + side at kb, its - side at ke) and
        // role 2 consumes them.  Interior planes: 5 rounds; roles 0-2 produce their
        // lines for the interior cells and consume the two lines of the round
        // that cross their faces, role 3 works on the ring cells.  Each kind
        // of wave runs its own loop (same barrier count), so the
        // accumulators never pass through a control-flow merge.
        const bool layer = (k == kb || k == ke);
        if (layer) {
            const bool bottom = k == kb;
#pragma unroll 1
            for (int r = 0; r < 3; r++) {
                LANE_GEOMETRY();
                const int t = role + 4 * r;
                double *pp = xch + role * PT * 64 + lane;
                if (t < 9) {
                    // the t-th z line through the cell: its + end lies on the
                    // cell's top face, its - end on the bottom face
                    const int dc = (int)(zline_dirs() >> (6 * t)) & 63;
                    const int dx = (dc & 3) - 1, dy = ((dc >> 2) & 3) - 1, dz = (dc >> 4) - 1;
                    const Line5 l = line5(ci, cj, k, dx, dy, dz);
                    CwW cw = {0.0, 0.0};
                    if (CW && (HYD || nspec > 0))
                        cw = cw_weights<VEL>(win, l, dx, dy, dz, gamma, gm1, de, cwmode, HYD);
                    if (HYD) {
                        if (bottom)
                            produce_hydro<true, false, VEL, CW>(win, l, pp, pp, gamma, gm1, de,
                                                                bits, cw);
                        else
                            produce_hydro<false, false, VEL, CW, true>(win, l, pp, pp, gamma, gm1,
                                                                       de, bits, cw);
                    } else if (nspec > 0) {
                        ppm_fields<CW, 6, NF_MAX>(win, l, cw, [&](int f, double qp, double qm) {
                            pp[f * 64] = bottom ? qp : qm;
                        });
                    }
                }
                lds_barrier();
                if (role == 2) {
                    // the round's points, all loaded before the first sum (the
                    // slots of idle producers hold older points, never summed)
                    constexpr uint32_t zw = zline_wcodes();
                    if (HYD) {
                        HPt q[4];
#pragma unroll
                        for (int w = 0; w < 4; w++) q[w] = load_h(xch + w * PT * 64 + lane, 2);
#pragma unroll
                        for (int w = 0; w < 4; w++) {
                            const int t2 = w + 4 * r;
                            if (t2 < 9)
                                acc_h_vals(acc[0], q[w].V, q[w].un, q[w].p, q[w].cs,
                                           simpson_wc((zw >> (2 * t2)) & 3));
                        }
                    } else {
                        SPt q[4];
#pragma unroll
                        for (int w = 0; w < 4; w++) q[w] = load_s(xch + w * PT * 64 + lane, 2);
#pragma unroll
                        for (int w = 0; w < 4; w++) {
                            const int t2 = w + 4 * r;
                            if (t2 < 9) acc_s_pt(acc[0], q[w], simpson_wc((zw >> (2 * t2)) & 3));
                        }
                    }
                }
                lds_barrier();
            }
        } else if (role < 3) {
            const int ax = role;
            const uint64_t ctab = ax == 0 ? cons_table(0) : ax == 1 ? cons_table(1) : cons_table(2);
            const uint64_t ptab = ax == 0 ? prod_table(0) : ax == 1 ? prod_table(1) : prod_table(2);
#pragma unroll 1
            for (int r = 0; r < 5; r++) {
                LANE_GEOMETRY();
                const int pd = (int)(ptab >> (7 * r)) & 127;
                double *pp = xch + (role * 2 + 0) * PT * 64 + lane;
                double *pm = xch + (role * 2 + 1) * PT * 64 + lane;
                if (pd & 64) {
                    const int dx = (pd & 3) - 1, dy = ((pd >> 2) & 3) - 1, dz = ((pd >> 4) & 3) - 1;
                    const Line5 l = line5(ci, cj, k, dx, dy, dz);
                    CwW cw = {0.0, 0.0};
                    if (CW && (HYD || nspec > 0))
                        cw = cw_weights<VEL>(win, l, dx, dy, dz, gamma, gm1, de, cwmode, HYD);
                    if (HYD) {
                        // and the last species field, to balance the pair (its
                        // values are loaded during the energy field; unused
                        // without species)
                        Pts5 xv;
                        produce_hydro<true, true, VEL, CW, false, NF_MAX - 1>(
                            win, l, pp, pm, gamma, gm1, de, bits, cw, &xv);
                        if (nspec > 0) {
                            double qp, qm;
                            ppm_pts<CW>(xv, NF_MAX - 1, cw, qp, qm);
                            pp[(NF_MAX - 1) * 64] = qp;
                            pm[(NF_MAX - 1) * 64] = qm;
                        }
                    } else if (nspec > 0) {
                        ppm_fields<CW, 6, NF_MAX - 1>(win, l, cw, [&](int f, double qp, double qm) {
                            pp[f * 64] = qp;
                            pm[f * 64] = qm;
                        });
                    }
                }
                lds_barrier();
                // the two lines of the round that cross my faces (one in the
                // last round: the second repeats the first with weight 0,
                // which leaves the sums and the speed extrema unchanged).
                // All four points are loaded before the first sum.
                {
                    const int d0 = (int)(ctab >> (10 * r)) & 31;
                    const int d1 = (int)(ctab >> (10 * r + 5)) & 31;
                    const double w0 = simpson_wc(d0 >> 3), w1 = simpson_wc(d1 >> 3);
                    const double *a0 = xch + (d0 & 7) * PT * 64 + lane;
                    const double *b0 = xch + ((d0 & 7) ^ 1) * PT * 64 + lane;
                    const double *a1 = xch + (d1 & 7) * PT * 64 + lane;
                    const double *b1 = xch + ((d1 & 7) ^ 1) * PT * 64 + lane;
                    if (HYD) {
                        const HPt pa0 = load_h(a0, ax), pb0 = load_h(b0, ax);
                        const HPt pa1 = load_h(a1, ax), pb1 = load_h(b1, ax);
                        acc_h_vals(acc[0], pa0.V, pa0.un, pa0.p, pa0.cs, w0);
                        acc_h_vals(acc[1], pb0.V, pb0.un, pb0.p, pb0.cs, w0);
                        acc_h_vals(acc[0], pa1.V, pa1.un, pa1.p, pa1.cs, w1);
                        acc_h_vals(acc[1], pb1.V, pb1.un, pb1.p, pb1.cs, w1);
                    } else {
                        const SPt pa0 = load_s(a0, ax), pb0 = load_s(b0, ax);
                        const SPt pa1 = load_s(a1, ax), pb1 = load_s(b1, ax);
                        acc_s_pt(acc[0], pa0, w0);
                        acc_s_pt(acc[1], pb0, w0);
                        acc_s_pt(acc[0], pa1, w1);
                        acc_s_pt(acc[1], pb1, w1);
                    }
                }
                lds_barrier();
            }
        } else {
#pragma unroll 1
            for (int r = 0; r < 5; r++) {
                LANE_GEOMETRY();
                // ring cell: 9 points of its face to the interior over two lanes
                // (t = 0..4 and 5..8; the second lane's last round repeats t = 8
                // with weight 0)
                const int t0 = half ? 5 + r : r;
                const int t = t0 < 9 ? t0 : 8;
                const double wt = t0 < 9 ? simpson_w(t % 3 - 1, t / 3 - 1) : 0.0;
                const int dn = r_side ? -1 : 1;    // normal component
                const int dx = r_axis == 0 ? dn : t % 3 - 1;
                const int dy = r_axis == 0 ? t % 3 - 1 : dn;
                const Line5 l = line5(ri, rj, k, dx, dy, t / 3 - 1);
                CwW cw = {0.0, 0.0};
                if (CW && (HYD || nspec > 0))
                    cw = cw_weights<VEL>(win, l, dx, dy, t / 3 - 1, gamma, gm1, de, cwmode, HYD);
                if (HYD) {
                    Pts5 xv;
                    const PlusState ps = produce_hydro<false, false, VEL, CW, false, NF_MAX - 1>(
                        win, l, nullptr, nullptr, gamma, gm1, de, bits, cw, &xv);
                    const double un = r_axis == 0 ? ps.vx : ps.vy;
                    acc_h_vals(acc[0], ps.q, un, ps.p, ps.cs, wt);
                    run[lane] = un;
                    if (nspec > 0) {
                        double qp, qm;
                        ppm_pts<CW>(xv, NF_MAX - 1, cw, qp, qm);
                        run[(NF_MAX - 1 - 5) * 64 + lane] = qp;
                    }
                } else if (nspec > 0) {
                    ppm_fields<CW, 6, NF_MAX - 1>(win, l, cw, [&](int f, double qp, double) {
                        run[(f - 5) * 64 + lane] = qp;
                    });
                }
                lds_barrier();
                if (!HYD) {
                    // ring species: the normal velocity came from the hydro wave
                    const double wun = wt * run[lane];
#pragma unroll
                    for (int i = 0; i < 5; i++) {
                        const double v = run[(1 + i) * 64 + lane];
                        acc[0][i] = fma(wt, v, acc[0][i]);
                        acc[0][5 + i] = fma(wun, v, acc[0][5 + i]);
                    }
                }
                lds_barrier();
            }
        }

        // plane k-2 is no longer read (the rounds' last barrier has passed):
        // its slot takes plane k+3 (prefetched one step ahead); then the loads
        // of plane k+4 start, behind this step's stores.  On interior planes
        // the barriers of the flux phases below order these stores before the
        // next step's reads; after the first face layer a barrier does.
        if (k + 3 <= ke + 2) {
            double *dst = win + ((k + 3) % SLOTS) * SLOT_D;
            if (VEL) {
#pragma unroll
                for (int q = 0; q < 2; q++)
                    if (mom[q]) pf[q] = pf[q] / pr[q];
            }
#pragma unroll
            for (int q = 0; q < 5; q++) dst[l_off[q]] = pf[q];
            if (k + 4 <= ke + 2) {
#pragma unroll
                for (int q = 0; q < 5; q++) pf[q] = *src(q, k + 4);
                if (VEL) {
#pragma unroll
                    for (int q = 0; q < 2; q++) pr[q] = *src_rho(q, k + 4);
                }
            }
        }
        if (layer) lds_barrier();

        if (layer) {
            LANE_GEOMETRY();
            if (k == kb) {
                if (role == 2 && work) {
                    if (HYD) store_h(zl + lane, 64, acc[0]);
                    else store_s(zl + lane, 64, acc[0]);
                }
            } else {
                // face (ke-1|ke): left partial from step ke-1, right = acc[0]; the
                // species wave gets the right-side speeds through LDS
                if (role == 2 && HYD) {
                    xch[ZB_OFF + 2 * 64 + lane] = acc[0][H_LP];
                    xch[ZB_OFF + 3 * 64 + lane] = acc[0][H_LM];
                }
                lds_barrier();
                if (role == 2 && work) {
                    double Fz[NF_MAX];
                    if (HYD) {
                        const Speeds sp = combine_h(acc[0], zl + lane, 64, false, 2, sym, Fz);
                        amax_l = fmax(amax_l, sp.amax_face);
                    } else {
                        const Speeds sp = face_speeds(zl[H_LP * 64 + lane], zl[H_LM * 64 + lane],
                                                      xch[ZB_OFF + 2 * 64 + lane],
                                                      xch[ZB_OFF + 3 * 64 + lane], sym);
                        combine_s(acc[0], zl + lane, 64, false, sp, Fz);
                    }
                    update_cell<VEL>(win, keep, lane, ke - 1, ci, cj, f0, f1, Fz, lam, rate,
                                     stg, Us, Os, fst, chk);
                }
            }
            continue;
        }

        // ---- face fluxes of plane k and the update of plane k-1
        {
        LANE_GEOMETRY();
        if (role == 3 && work) {
            // the two lanes of a ring cell hold partial sums: add them
#pragma unroll
            for (int i = 0; i < NH; i++) {
                const double o = pair_swap(acc[0][i]);
                if (HYD && i == H_LP) acc[0][i] = fmax(acc[0][i], o);
                else if (HYD && i == H_LM) acc[0][i] = fmin(acc[0][i], o);
                else acc[0][i] += o;
            }
        }
        // phase 1: right-side partials and left-side speeds -> LDS
        if ((role == 0 || role == 1) && work) {
            double *R = xch + XR_OFF + (role == 0 ? (0 * 8 + (cj - 3)) * 9 + (ci - 3)
                                                  : (1 * 8 + (ci - 3)) * 9 + (cj - 3));
            if (HYD) store_h(R, RST, acc[1]);
            else store_s(R, RST, acc[1]);
        }
        if (role == 3 && half == 0 && r_side == 1 && work) {
            double *R = xch + XR_OFF + (r_axis * 8 + (r_pos - 3)) * 9 + 8;
            if (HYD) store_h(R, RST, acc[0]);
            else store_s(R, RST, acc[0]);
        }
        if (HYD) {
            int ll = -1;
            if (role == 0) ll = (0 * 8 + (cj - 3)) * 9 + (ci - 2);
            if (role == 1) ll = (1 * 8 + (ci - 3)) * 9 + (cj - 2);
            if (role == 3 && half == 0 && r_side == 0) ll = (r_axis * 8 + (r_pos - 3)) * 9;
            if (ll >= 0) {
                xch[LL_OFF + ll] = acc[0][H_LP];
                xch[LL_OFF + RST + ll] = acc[0][H_LM];
            }
            if (role == 2) {   // z face (k-1|k): left speeds (last step), right speeds
                xch[ZB_OFF + 0 * 64 + lane] = zl[H_LP * 64 + lane];
                xch[ZB_OFF + 1 * 64 + lane] = zl[H_LM * 64 + lane];
                xch[ZB_OFF + 2 * 64 + lane] = acc[1][H_LP];
                xch[ZB_OFF + 3 * 64 + lane] = acc[1][H_LM];
            }
        }
        lds_barrier();
        // phase 2: left owners form the x/y face fluxes; z owners the z face
        if (work && (role < 2 || (role == 3 && half == 0 && r_side == 0))) {
            const int ax = role < 2 ? role : r_axis;
            const int row = role == 0 ? cj - 3 : role == 1 ? ci - 3 : r_pos - 3;
            const int p = role == 0 ? ci - 2 : role == 1 ? cj - 2 : 0;
            const int fi = (ax * 8 + row) * 9 + p;
            const double *R = xch + XR_OFF + fi;
            double *Fo = xch + XF_OFF + fi;
            if (HYD) {
                const Speeds sp = combine_h(acc[0], R, RST, true, ax, sym, Fb);
                amax_l = fmax(amax_l, sp.amax_face);
            } else {
                const Speeds sp = face_speeds(xch[LL_OFF + fi], xch[LL_OFF + RST + fi],
                                              R[H_LP * RST], R[H_LM * RST], sym);
                combine_s(acc[0], R, RST, true, sp, Fb);
            }
#pragma unroll
            for (int f = 0; f < NF_MAX; f++)
                if (f >= f0 && f < f1x) Fo[f * RST] = Fb[f];
        }
        if (role == 2 && work) {
            // z-face (k-1|k): left partial from the previous step, right = acc[1]
            double Fz[NF_MAX];
            if (HYD) {
                const Speeds sp = combine_h(acc[1], zl + lane, 64, false, 2, sym, Fz);
                amax_l = fmax(amax_l, sp.amax_face);
            } else {
                const Speeds sp = face_speeds(xch[ZB_OFF + lane], xch[ZB_OFF + 64 + lane],
                                              xch[ZB_OFF + 128 + lane], xch[ZB_OFF + 192 + lane],
                                              sym);
                combine_s(acc[1], zl + lane, 64, false, sp, Fz);
            }
            // plane k-1's summed flux differences (its cells are written after
            // the barrier, where the x owner overwrites the kept x/y part)
#pragma unroll
            for (int f = 0; f < NF_MAX; f++)
                if (f >= f0 && f < f1x) {
                    dsum[f] = keep[(NF_MAX + f) * 64 + lane] + (Fz[f] - keep[f * 64 + lane]);
                    keep[f * 64 + lane] = Fz[f];
                }
            if (HYD) store_h(zl + lane, 64, acc[0]);
            else store_s(zl + lane, 64, acc[0]);
        }
        lds_barrier();
        // phase 3: the x owner forms its cells' x/y flux difference,
        // (F_x right - F_x left) + (F_y above - F_y below), the x fluxes from
        // its own right face and the face array, the y fluxes from the face
        // array.  The first round of the next step writes only below XF_OFF,
        // and the z-line producer (which writes above it) first produces in
        // the second round, after the first round's barriers, so no barrier
        // is needed here.
        if (role == 2 && k >= kb + 2 && work)
            update_cell_sum<VEL>(win, k - 1, ci, cj, f0, f1, dsum, lam, rate, stg, Us, Os, fst,
                                 chk);
        if (role == 0 && work) {
            const double *Fl = xch + XF_OFF + (cj - 3) * 9 + (ci - 3);     // left x face
            const double *Fy = xch + XF_OFF + (8 + (ci - 3)) * 9 + (cj - 3); // y face below
#pragma unroll
            for (int f = 0; f < NF_MAX; f++)
                if (f >= f0 && f < f1x)
                    keep[(NF_MAX + f) * 64 + lane] =
                        (Fb[f] - Fl[f * RST]) + (Fy[f * RST + 1] - Fy[f * RST]);
        }
        }
    }
    if (chk != chk) bits |= HYDRO_STATUS_NONFINITE;

}

// ---- subgrids without species: two planes at a time ---------------------------
//
// A subgrid without species leaves the species wave of every role idle.  The
// paired body splits the eight waves into two groups of four roles: group 0
// (the first wave of each role) runs the plane schedule above on plane k,
// group 1 (the second wave) on plane k + 1, so every SIMD carries two hydro
// waves, and a step advances two planes.  Each group's sums keep the order of
// the 11-field plan and every formula rounds as there, so the results are the
// same bits.  It lives in a kernel instance of its own, beside the 11-field
// body for the other subgrids; batches known to hold no subgrid without
// species get the instance without it, whose registers it would crowd.
// The LDS plan (in doubles):
//   a window of 6 planes of the 6 hydro fields (planes k-2 .. k+3), one
//   exchange area per group with 11-double points (V[0..5], v, p, c) and the
//   group's flux-phase arrays inside it, the z partial carried to the next
//   step (group 1 -> group 0) and the one passed within a step (group 0 ->
//   group 1), and each group's z fluxes and x/y differences, kept for two
//   steps (by the step's parity).
// A plane's cells are updated once both of its z fluxes exist: plane k-2 (all
// of whose terms are the last step's) by group 1's z owner in the first flux
// phase, plane k-1 by group 0's z owner in the second, right after it forms
// that plane's upper flux.  Nothing is carried in registers from one step to
// the next but the window's prefetched planes.  The 9 z lines of a face
// layer are produced by all eight waves and summed by group 0's z owner.
namespace pr {
constexpr int SL = 6;                       // window planes
constexpr int SD = 6 * NPLANE + 2;          // one window plane, + a dummy word
constexpr int WIN = SL * SD;
constexpr int VX = 6;                       // point: V[0..5], vx, vy, vz, p, c
constexpr int SLOT = 11 * 64;
constexpr int XG = 6 * SLOT;                // one group's exchange area
constexpr int XR = 0;                       // [NH][2][8][9] right partials
constexpr int LL = NH * RST;                // [2][2][8][9] left speeds
constexpr int XF = 4 * SLOT;                // [6][2][8][9] face fluxes
constexpr int X0 = WIN;                     // group g's area at X0 + g XG
constexpr int ZL = X0 + 2 * XG;             // [NH][64]
constexpr int ZX = ZL + NH * 64;            // [NH][64]
constexpr int FZ = ZX + NH * 64;            // [parity][group][6][64] z fluxes
constexpr int KP = FZ + 4 * 6 * 64;         // [parity][group][6][64] x/y differences
constexpr int END = KP + 4 * 6 * 64;
// offsets of field f of group g's z fluxes and x/y differences of step parity par
__device__ __forceinline__ int fz(int par, int g, int f) {
    return FZ + ((par * 2 + g) * 6 + f) * 64;
}
__device__ __forceinline__ int kp(int par, int g, int f) {
    return KP + ((par * 2 + g) * 6 + f) * 64;
}
static_assert(LL + 2 * RST <= XF && XF + 6 * RST <= XG, "a group's flux arrays");
static_assert(4 * SLOT <= XF, "round 0 writes below the face fluxes (slots of roles 0 and 1)");
static_assert(END * 8 + 512 <= 163840, "paired LDS plan");
static_assert(6 * NPLANE <= 3 * NT, "a plane of 6 fields in three elements per thread");

__device__ __forceinline__ Line5 line5(int i, int j, int k, int dx, int dy, int dz) {
    Line5 l;
#pragma unroll
    for (int m = -2; m <= 2; m++) {
        const int pl = (k + m * dz) % SL;
        l.o[m + 2] = pl * SD + (j + m * dy) * NB + (i + m * dx);
    }
    return l;
}

// The update of plane kc's cell (ci, cj) of the window: its x/y difference at
// lds + d, the upper z fluxes Fu and the lower at lds + fl (fields 64 apart),
// summed in the order of the 11-field plan.
__device__ __forceinline__ void update_w(const double *lds, int kc, int ci, int cj, int lane,
                                         int d, const double *Fu, int fl, double lam, bool rate,
                                         const Stage &stg, double *Os, int fst, double &chk) {
    const int cidx = opaque_v(kc * GNP + cj * GNB + ci);
    double vv[6];
#pragma unroll
    for (int f = 0; f < 6; f++) {
        const double u = lds[(kc % SL) * SD + f * NPLANE + cj * NB + ci];
        const double dfz = Fu[f] - lds[fl + f * 64 + lane];
        const double sxy = lds[d + f * 64 + lane];
        vv[f] = (rate ? 0.0 : u) - lam * (sxy + dfz);
    }
#pragma unroll
    for (int f = 0; f < 6; f++) {
        double v = vv[f];
        if (stg.U0) {
            const double u0 = stg.U0[f * fst + cidx];
            v = stg.identity ? u0 : fma(stg.c0, u0, stg.c1 * v);
        }
        chk = fma(v, 0.0, chk);
        Os[f * fst + cidx] = v;
    }
}
}  // namespace pr

struct PairOut {
    double amax;
    int bits;
};

// what the ghost map's check reads from the launch's arguments
struct PairMeta {
    const int32_t *gsrc, *gmode, *n_species;
    const int64_t *offset;
    int32_t n_sub;
};

template <bool GATHER>
__device__ __forceinline__ PairOut subgrid_pair(
    double *lds, int tid, int role, int grp, const double *Us0, double *Os0, int fst0, double lam,
    bool rate, Stage stg, bool sym, double gamma, double gm1, double de, PairMeta a, int s,
    const double *Ug, int64_t *toff, int *tmode, int kb_, int ke_) {
    // uniform values as scalars, so that branches and addresses derived from
    // them stay scalar
    role = __builtin_amdgcn_readfirstlane(role);
    grp = __builtin_amdgcn_readfirstlane(grp);
    fst0 = __builtin_amdgcn_readfirstlane(fst0);
    s = __builtin_amdgcn_readfirstlane(s);
    const int kb = __builtin_amdgcn_readfirstlane(kb_), ke = __builtin_amdgcn_readfirstlane(ke_);
    double *win = lds;
    double *xg = lds + pr::X0 + grp * pr::XG;
    double *zl = lds + pr::ZL;
    double *zx = lds + pr::ZX;
    double amax_l = 0.0;
    int bits = 0;
    double chk = 0.0;
    constexpr int nspec = 0;
    int g_off[3], l_off[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        const int e = tid + q * NT;
        const int f = e / NPLANE, c = e - f * NPLANE;
        const bool ok = e < 6 * NPLANE;
        if (!GATHER) {
            g_off[q] = ok ? f * fst0 + GCELL(c) : 0;
        } else {
            const int i = ok ? c % NB : NG, j = ok ? c / NB : NG;
            const int dx = i < NG ? -1 : (i >= NG + NSUB ? 1 : 0);
            const int dy = j < NG ? -1 : (j >= NG + NSUB ? 1 : 0);
            g_off[q] = i | (j << 4) | ((dx + 1) << 8) | ((dy + 1) << 10) | ((ok ? f : 0) << 12);
        }
        l_off[q] = ok ? f * NPLANE + c : 6 * NPLANE;
    }
    auto src = [&](int q, int pk) -> const double * {
        if (!GATHER) return Us0 + (g_off[q] + pk * GNP);
        const int g = opaque_v(g_off[q]);
        return gather_ptr(Ug, toff, tmode, (g >> 12) * fst0, g, pk);
    };

    lds_barrier();   // the previous subgrid's LDS reads are done
    if (GATHER) {
        if (tid < 27) {
            const int64_t own = Us0 - Ug;
            int64_t o = own;
            int m = tid == 13 ? 0 : 7;
            if (tid != 13) {
                const int sb = a.gsrc[s * 27 + tid];
                bool good = sb >= 0 && sb < a.n_sub;
                if (good) {
                    const int ns2 = a.n_species[sb];
                    const int64_t o2 = a.offset[sb];
                    good = ns2 >= 0 && ns2 <= 5 && ns2 >= nspec && o2 >= 0 && !(o2 & 1);
                    if (good) {
                        o = o2;
                        m = a.gmode[s * 27 + tid];
                    }
                }
                if (!good) bits |= HYDRO_STATUS_BADMETA;
            }
            toff[tid] = o;
            tmode[tid] = m;
        }
        lds_barrier();
    }
    // window: planes kb-2 .. kb+3; then planes kb+4 (after the lower face
    // layer) and kb+5 are held in registers
    {
        double v[pr::SL][3];
#pragma unroll
        for (int pl = 0; pl < pr::SL; pl++)
#pragma unroll
            for (int q = 0; q < 3; q++) v[pl][q] = *src(q, kb - 2 + pl);
#pragma unroll
        for (int pl = 0; pl < pr::SL; pl++) {
            double *dst = win + ((kb - 2 + pl) % pr::SL) * pr::SD;
#pragma unroll
            for (int q = 0; q < 3; q++) dst[l_off[q]] = v[pl][q];
        }
    }
    double pf[2][3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
        pf[0][q] = kb + 4 <= ke + 2 ? *src(q, kb + 4) : 0.0;
        pf[1][q] = kb + 5 <= ke + 2 ? *src(q, kb + 5) : 0.0;
    }
    lds_barrier();

    double acc[2][NH];
    double Fb[6];
    const CwW cw0 = {0.0, 0.0};
    int par = 0;         // parity of the pair step: its z fluxes and x/y differences
    for (int k = kb; k <= ke;) {
        const bool layer = (k == kb || k == ke);
        acc_zero(acc[0], true);
        acc_zero(acc[1], true);
        if (layer) {
            // the 9 z lines of the face layer in one round: lines 0-7 by the
            // eight waves, line 8 also by group 0's z owner (into a free slot
            // of group 1's area), which then sums them in line order
            const bool bottom = k == kb;
            constexpr uint32_t zw = zline_wcodes();
            {
                LANE_GEOMETRY();
                const bool zo = role == 2 && grp == 0;
                double *x8 = lds + pr::X0 + pr::XG + 4 * pr::SLOT + lane;
#pragma unroll 1
                for (int u = 0; u < (zo ? 2 : 1); u++) {
                    const int t = u == 0 ? role + 4 * grp : 8;
                    double *pp = u == 0 ? xg + role * pr::SLOT + lane : x8;
                    const int dc = (int)(zline_dirs() >> (6 * t)) & 63;
                    const int dx = (dc & 3) - 1, dy = ((dc >> 2) & 3) - 1, dz = (dc >> 4) - 1;
                    const Line5 l = pr::line5(ci, cj, k, dx, dy, dz);
                    if (bottom)
                        produce_hydro<true, false, false, false, false, -1, pr::VX>(
                            win, l, pp, pp, gamma, gm1, de, bits, cw0);
                    else
                        produce_hydro<false, false, false, false, true, -1, pr::VX>(
                            win, l, pp, pp, gamma, gm1, de, bits, cw0);
                }
                lds_barrier();
                if (zo) {
#pragma unroll 1
                    for (int g = 0; g < 2; g++) {
                        const double *xs = lds + pr::X0 + g * pr::XG + lane;
                        HPt q[4];
#pragma unroll
                        for (int w = 0; w < 4; w++) q[w] = load_h<pr::VX>(xs + w * pr::SLOT, 2);
#pragma unroll
                        for (int w = 0; w < 4; w++)
                            acc_h_vals(acc[0], q[w].V, q[w].un, q[w].p, q[w].cs,
                                       simpson_wc((zw >> (2 * (w + 4 * g))) & 3));
                    }
                    const HPt q8 = load_h<pr::VX>(x8, 2);
                    acc_h_vals(acc[0], q8.V, q8.un, q8.p, q8.cs, simpson_wc((zw >> 16) & 3));
                }
            }
            LANE_GEOMETRY();
            if (bottom) {
                // plane kb+4 into the slot of kb-2; kb+5 moves up, kb+6 is loaded
                if (kb + 4 <= ke + 2) {
                    double *dst = win + ((kb + 4) % pr::SL) * pr::SD;
#pragma unroll
                    for (int q = 0; q < 3; q++) dst[l_off[q]] = pf[0][q];
                }
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    pf[0][q] = pf[1][q];
                    pf[1][q] = kb + 6 <= ke + 2 ? *src(q, kb + 6) : 0.0;
                }
                if (role == 2 && grp == 0) store_h(zl + lane, 64, acc[0]);
                lds_barrier();
                k += 1;
            } else {
                // face (ke-1|ke), its left partial from the last pair step's
                // group 1; planes ke-2 and ke-1 are updated
                const int pl = par ^ 1;
                if (role == 2 && grp == 1 && ke - 2 >= kb + 1) {
                    double Fu[6];
#pragma unroll
                    for (int f = 0; f < 6; f++) Fu[f] = lds[pr::fz(pl, 1, f) + lane];
                    pr::update_w(lds, ke - 2, ci, cj, lane, pr::kp(pl, 0, 0), Fu, pr::fz(pl, 0, 0),
                                 lam, rate, stg, Os0, fst0, chk);
                }
                if (role == 2 && grp == 0) {
                    double Fz[6];
                    const Speeds sp = combine_h(acc[0], zl + lane, 64, false, 2, sym, Fz);
                    amax_l = fmax(amax_l, sp.amax_face);
                    if (ke - 1 >= kb + 1)
                        pr::update_w(lds, ke - 1, ci, cj, lane, pr::kp(pl, 1, 0), Fz,
                                     pr::fz(pl, 1, 0), lam, rate, stg, Os0, fst0, chk);
                }
                k += 1;
            }
            continue;
        }

        // ---- a pair step: plane k by group 0, plane k+1 by group 1
        const int kg = k + grp;
        const int pl = par ^ 1;      // the last pair step's buffers
        if (role < 3) {
            const int ax = role;
            const uint64_t ctab = ax == 0 ? cons_table(0) : ax == 1 ? cons_table(1) : cons_table(2);
            const uint64_t ptab = ax == 0 ? prod_table(0) : ax == 1 ? prod_table(1) : prod_table(2);
#pragma unroll 1
            for (int r = 0; r < 5; r++) {
                LANE_GEOMETRY();
                const int pd = (int)(ptab >> (7 * r)) & 127;
                if (pd & 64) {
                    const int dx = (pd & 3) - 1, dy = ((pd >> 2) & 3) - 1, dz = ((pd >> 4) & 3) - 1;
                    const Line5 l = pr::line5(ci, cj, kg, dx, dy, dz);
                    produce_hydro<true, true, false, false, false, -1, pr::VX>(
                        win, l, xg + (role * 2 + 0) * pr::SLOT + lane,
                        xg + (role * 2 + 1) * pr::SLOT + lane, gamma, gm1, de, bits, cw0);
                }
                lds_barrier();
                {
                    const int d0 = (int)(ctab >> (10 * r)) & 31;
                    const int d1 = (int)(ctab >> (10 * r + 5)) & 31;
                    const double w0 = simpson_wc(d0 >> 3), w1 = simpson_wc(d1 >> 3);
                    const HPt pa0 = load_h<pr::VX>(xg + (d0 & 7) * pr::SLOT + lane, ax);
                    const HPt pb0 = load_h<pr::VX>(xg + ((d0 & 7) ^ 1) * pr::SLOT + lane, ax);
                    const HPt pa1 = load_h<pr::VX>(xg + (d1 & 7) * pr::SLOT + lane, ax);
                    const HPt pb1 = load_h<pr::VX>(xg + ((d1 & 7) ^ 1) * pr::SLOT + lane, ax);
                    acc_h_vals(acc[0], pa0.V, pa0.un, pa0.p, pa0.cs, w0);
                    acc_h_vals(acc[1], pb0.V, pb0.un, pb0.p, pb0.cs, w0);
                    acc_h_vals(acc[0], pa1.V, pa1.un, pa1.p, pa1.cs, w1);
                    acc_h_vals(acc[1], pb1.V, pb1.un, pb1.p, pb1.cs, w1);
                }
                lds_barrier();
            }
        } else {
#pragma unroll 1
            for (int r = 0; r < 5; r++) {
                LANE_GEOMETRY();
                const int t0 = half ? 5 + r : r;
                const int t = t0 < 9 ? t0 : 8;
                const double wt = t0 < 9 ? simpson_w(t % 3 - 1, t / 3 - 1) : 0.0;
                const int dn = r_side ? -1 : 1;
                const int dx = r_axis == 0 ? dn : t % 3 - 1;
                const int dy = r_axis == 0 ? t % 3 - 1 : dn;
                const Line5 l = pr::line5(ri, rj, kg, dx, dy, t / 3 - 1);
                const PlusState ps = produce_hydro<false, false, false, false>(
                    win, l, nullptr, nullptr, gamma, gm1, de, bits, cw0);
                acc_h_vals(acc[0], ps.q, r_axis == 0 ? ps.vx : ps.vy, ps.p, ps.cs, wt);
                lds_barrier();
                lds_barrier();
            }
        }

        LANE_GEOMETRY();
        if (role == 3) {
#pragma unroll
            for (int i = 0; i < NH; i++) {
                const double o = pair_swap(acc[0][i]);
                if (i == H_LP) acc[0][i] = fmax(acc[0][i], o);
                else if (i == H_LM) acc[0][i] = fmin(acc[0][i], o);
                else acc[0][i] += o;
            }
        }
        // phase 1: right partials and left speeds of the group's x/y faces;
        // group 0's z owner passes its upper partial to group 1; group 1's z
        // owner updates plane k-2 (all its terms are the last step's)
        if (role == 0 || role == 1) {
            double *R = xg + pr::XR + (role == 0 ? (0 * 8 + (cj - 3)) * 9 + (ci - 3)
                                                 : (1 * 8 + (ci - 3)) * 9 + (cj - 3));
            store_h(R, RST, acc[1]);
        }
        if (role == 3 && half == 0 && r_side == 1) {
            double *R = xg + pr::XR + (r_axis * 8 + (r_pos - 3)) * 9 + 8;
            store_h(R, RST, acc[0]);
        }
        {
            int ll = -1;
            if (role == 0) ll = (0 * 8 + (cj - 3)) * 9 + (ci - 2);
            if (role == 1) ll = (1 * 8 + (ci - 3)) * 9 + (cj - 2);
            if (role == 3 && half == 0 && r_side == 0) ll = (r_axis * 8 + (r_pos - 3)) * 9;
            if (ll >= 0) {
                xg[pr::LL + ll] = acc[0][H_LP];
                xg[pr::LL + RST + ll] = acc[0][H_LM];
            }
        }
        if (role == 2 && grp == 0) store_h(zx + lane, 64, acc[0]);
        if (role == 2 && grp == 1 && k - 2 >= kb + 1) {
            double Fu[6];
#pragma unroll
            for (int f = 0; f < 6; f++) Fu[f] = lds[pr::fz(pl, 1, f) + lane];
            pr::update_w(lds, k - 2, ci, cj, lane, pr::kp(pl, 0, 0), Fu, pr::fz(pl, 0, 0), lam,
                         rate, stg, Os0, fst0, chk);
        }
        lds_barrier();
        // phase 2: x/y face fluxes; the z faces (k-1|k) (group 0, which then
        // updates plane k-1) and (k|k+1) (group 1)
        if (role < 2 || (role == 3 && half == 0 && r_side == 0)) {
            const int ax = role < 2 ? role : r_axis;
            const int row = role == 0 ? cj - 3 : role == 1 ? ci - 3 : r_pos - 3;
            const int p = role == 0 ? ci - 2 : role == 1 ? cj - 2 : 0;
            const int fi = (ax * 8 + row) * 9 + p;
            const Speeds sp = combine_h(acc[0], xg + pr::XR + fi, RST, true, ax, sym, Fb);
            amax_l = fmax(amax_l, sp.amax_face);
#pragma unroll
            for (int f = 0; f < 6; f++) xg[pr::XF + fi + f * RST] = Fb[f];
        }
        if (role == 2) {
            double Fz[6];
            const Speeds sp = combine_h(acc[1], (grp == 0 ? zl : zx) + lane, 64, false, 2, sym, Fz);
            amax_l = fmax(amax_l, sp.amax_face);
#pragma unroll
            for (int f = 0; f < 6; f++) lds[pr::fz(par, grp, f) + lane] = Fz[f];
            if (grp == 0 && k - 1 >= kb + 1)
                pr::update_w(lds, k - 1, ci, cj, lane, pr::kp(pl, 1, 0), Fz, pr::fz(pl, 1, 0), lam,
                             rate, stg, Os0, fst0, chk);
        }
        lds_barrier();
        // phase 3: each group's x owner forms its plane's x/y difference;
        // group 1 passes its upper partial to the next step; the two planes
        // after the window are stored
        if (role == 2 && grp == 1) store_h(zl + lane, 64, acc[0]);
        if (role == 0) {
            const double *Fl = xg + pr::XF + (cj - 3) * 9 + (ci - 3);
            const double *Fy = xg + pr::XF + (8 + (ci - 3)) * 9 + (cj - 3);
#pragma unroll
            for (int f = 0; f < 6; f++)
                lds[pr::kp(par, grp, f) + lane] =
                    (Fb[f] - Fl[f * RST]) + (Fy[f * RST + 1] - Fy[f * RST]);
        }
        if (k + 4 <= ke + 2) {
            double *dst = win + ((k + 4) % pr::SL) * pr::SD;
#pragma unroll
            for (int q = 0; q < 3; q++) dst[l_off[q]] = pf[0][q];
        }
        if (k + 5 <= ke + 2) {
            double *dst = win + ((k + 5) % pr::SL) * pr::SD;
#pragma unroll
            for (int q = 0; q < 3; q++) dst[l_off[q]] = pf[1][q];
        }
#pragma unroll
        for (int q = 0; q < 3; q++) {
            pf[0][q] = k + 6 <= ke + 2 ? *src(q, k + 6) : 0.0;
            pf[1][q] = k + 7 <= ke + 2 ? *src(q, k + 7) : 0.0;
        }
        lds_barrier();
        par ^= 1;
        k += 2;
    }
    if (chk != chk) bits |= HYDRO_STATUS_NONFINITE;
    PairOut out;
    out.amax = amax_l;
    out.bits = bits;
    return out;
}

// ---- the kernel ---------------------------------------------------------------

// Scratch of the split and dynamic launch shapes (32-bit words): [0] next work
// item, [1] workgroups done, [16, 16 + 2 n) per-subgrid running max of the
// parts' face speeds (as 64-bit patterns of non-negative doubles), then n
// status words and n arrival counts.  Every word is back at zero when the
// launch ends (the last workgroup or part to finish clears what it used).
__device__ __forceinline__ unsigned long long *sc_amax(uint32_t *sc) {
    return reinterpret_cast<unsigned long long *>(sc + 16);
}
__device__ __forceinline__ uint32_t *sc_bits(uint32_t *sc, int n) { return sc + 16 + 2 * n; }
__device__ __forceinline__ uint32_t *sc_count(uint32_t *sc, int n) { return sc + 16 + 3 * n; }

// LDS of an instance: the paired body's plan is the larger
constexpr int lds_doubles(bool pair) { return pair && pr::END > LDS_D ? pr::END : LDS_D; }

// PAIR: the instance that also holds the paired body, which sweeps the
// subgrids without species when their parts hold at least two planes.
template <bool VEL, bool CW, bool GATHER, bool PAIR = false>
__global__ __launch_bounds__(NT, 2) void k_fused(FusedArgs a, const double *__restrict__ U,
                                                 double *Uo,
                                                 double *__restrict__ amax,
                                                 int32_t *__restrict__ status, int order) {
    __shared__ double lds[lds_doubles(PAIR)];
    __shared__ double red_pair[PAIR ? 8 : 1];
    __shared__ int red_bits[8];
    __shared__ int next_item[2];     // by parity of the iteration (no barrier between
                                     // one iteration's read and the next one's write)
    __shared__ int64_t g_toff[GATHER ? 27 : 1];    // ghost-map table of the current subgrid
    __shared__ int g_tmode[GATHER ? 27 : 1];
    double *win = lds;
    double *xch = lds + WIN_D;
    double *zl = xch + XCH_D;          // z-face left partials carried between steps
    double *keep = zl + ZL_D;          // [0: F_z of the face below][1: dFx+dFy][11][64]
    double *run = keep + KEEP_D;       // ring lanes' normal velocity
    double *red = PAIR ? red_pair : run + RUN_D;

    // the role as a scalar: branches on it are then uniform branches, with no
    // exec-mask bookkeeping.  (The field-group test stays a vector compare: as
    // a scalar it made the allocator spill 108 bytes per lane instead of none.)
    const int tid = threadIdx.x, wave = tid >> 6;
    const int role = __builtin_amdgcn_readfirstlane(wave) & 3;
    const bool hyd = wave < 4;

    const double gamma = a.gamma, gm1 = a.gamma - 1.0, de = a.de_switch;
    const bool rate = a.rate != 0;
    const bool sym = a.sym != 0;
    const int cwmode = (a.steepen ? 1 : 0) | (a.flatten ? 2 : 0);
    // work items: the parts of the subgrids' z sweeps (P parts of 8 / P
    // interior planes each, part q of subgrid s is item s P + q), fetched in
    // a static stride or, in the dynamic form, from a counter in scratch
    const int lp = a.log_parts, P = 1 << lp, span = NSUB >> lp;
    const int n_items = a.n_sub << lp;
    uint32_t *sc = a.scratch;

    int parity = 0;
    for (int it = blockIdx.x; it < n_items; parity ^= 1) {
        const int s0 = it >> lp, q = it & (P - 1);
        const int s = order ? (a.n_sub - 1 - s0) : s0;
        const int kb = NG - 1 + q * span, ke = kb + span + 1;
        const int nspec = a.n_species[s];
        const int64_t off = a.offset[s];
        const int64_t ooff = a.out_offset ? a.out_offset[s] : off;
        const bool bad = nspec < 0 || nspec > 5 || off < 0 || (off & 1) || ooff < 0 || (ooff & 1);
        double amax_l = 0.0;
        int bits = 0;
        if (!bad) {
            const double dtv = a.clock ? a.clock[1] : a.dt;
            const double lam = rate ? 1.0 / a.h[s] : dtv / a.h[s];
            Stage stg;
            stg.U0 = a.U0 ? a.U0 + off : nullptr;
            stg.c0 = a.c0;
            stg.c1 = a.c1;
            stg.identity = dtv == 0.0;
            const double *Us0 = U + off;
            double *Os0 = Uo + ooff;
            const int fst0 = a.fstride;
            if (PAIR && nspec == 0 && span >= 2) {
                PairMeta pm;
                pm.gsrc = a.gsrc;
                pm.gmode = a.gmode;
                pm.n_species = a.n_species;
                pm.offset = a.offset;
                pm.n_sub = a.n_sub;
                const PairOut po = subgrid_pair<GATHER>(
                    lds, tid, role, __builtin_amdgcn_readfirstlane(wave) >> 2, Us0, Os0, fst0,
                    lam, rate, stg, sym, gamma, gm1, de, pm, s, U, g_toff, g_tmode, kb, ke);
                amax_l = po.amax;
                bits = po.bits;
            } else if (hyd) {
                subgrid_body<true, VEL, CW, GATHER>(win, xch, zl, keep, run, tid, role, nspec, Us0,
                                                    Os0, fst0, lam, rate, stg, sym, cwmode, gamma,
                                                    gm1, de, amax_l, bits, a, s, U, g_toff,
                                                    g_tmode, kb, ke);
            } else {
                subgrid_body<false, VEL, CW, GATHER>(win, xch, zl, keep, run, tid, role, nspec,
                                                     Us0, Os0, fst0, lam, rate, stg, sym, cwmode,
                                                     gamma, gm1, de, amax_l, bits, a, s, U, g_toff,
                                                     g_tmode, kb, ke);
            }

            // ---- the part's speed and status
            for (int o = 32; o > 0; o >>= 1) {
                amax_l = fmax(amax_l, __shfl_xor(amax_l, o));
                bits |= __shfl_xor(bits, o);
            }
            if ((tid & 63) == 0) {
                red[wave] = amax_l;
                red_bits[wave] = bits;
            }
        }
        if (a.dyn && tid == 0)
            next_item[parity] = (int)gridDim.x + (int)atomicAdd(&sc[0], 1u);
        lds_barrier();
        if (tid == 0) {
            double m = 0.0;
            int b = HYDRO_STATUS_BADMETA;
            if (!bad) {
                b = 0;
                for (int w = 0; w < 8; w++) {
                    m = fmax(m, red[w]);
                    b |= red_bits[w];
                }
            }
            bool last = true;
            if (P > 1) {
                // the last part of the subgrid to arrive writes its result
                atomicMax(&sc_amax(sc)[s], (unsigned long long)__double_as_longlong(m));
                atomicOr(&sc_bits(sc, a.n_sub)[s], (uint32_t)b);
                __threadfence();
                last = atomicAdd(&sc_count(sc, a.n_sub)[s], 1u) == (uint32_t)(P - 1);
                if (last) {
                    __threadfence();
                    m = __longlong_as_double(
                        (long long)atomicExch(&sc_amax(sc)[s], 0ull));
                    b = (int)atomicExch(&sc_bits(sc, a.n_sub)[s], 0u);
                    atomicExch(&sc_count(sc, a.n_sub)[s], 0u);
                }
            }
            if (last) {
                if (!isfinite(m)) b |= HYDRO_STATUS_NONFINITE;
                amax[s] = m;
                if (status) status[s] = (rate || a.U0) ? (status[s] | b) : b;
            }
        }
        it = a.dyn ? next_item[parity] : it + (int)gridDim.x;
    }
    if (a.dyn) {
        // the last workgroup out clears the counters for the next launch
        if (tid == 0) {
            __threadfence();
            if (atomicAdd(&sc[1], 1u) == gridDim.x - 1) {
                atomicExch(&sc[0], 0u);
                atomicExch(&sc[1], 0u);
            }
        }
    }
}

struct Variant {
    const char *name;
    int grid_per_cu;   // persistent workgroups per CU; 0 = one workgroup per work item
    int order;         // 0: subgrid order, 1: reverse order
    int log_parts;     // each subgrid's z sweep in 2^log_parts parts (work items)
    int dyn;           // work items fetched from a counter instead of a static stride
};

// The launch shapes the autotuner chooses from.  A part of a subgrid sweeps
// 8 / P interior planes plus the face layer below and above them, so P parts
// cost more in all than one sweep, but spread a batch of fewer subgrids than
// CUs over more of the chip.
constexpr Variant kVariants[] = {
    {"persistent-1x", 1, 0, 0, 0},
    {"persistent-2x", 2, 0, 0, 0},
    {"one-per-subgrid", 0, 0, 0, 0},
    {"persistent-1x-rev", 1, 1, 0, 0},
    {"persistent-1x-dynamic", 1, 0, 0, 1},
    {"split-2", 0, 0, 1, 0},
    {"split-4", 0, 0, 2, 0},
    {"split-8", 0, 0, 3, 0},
};
constexpr int kVariantSplit2 = 5;
static_assert(kVariants[kVariantSplit2].log_parts == 1 &&
                  kVariants[kVariantSplit2 + 2].log_parts == 3,
              "split variants in order");

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cus = 256;
    }
    return cus;
}

// The instantiation for the call's options: velocity reconstruction and the
// Colella-Woodward weights each have their own kernel, so the default one
// carries neither.
using FusedKernel = void (*)(FusedArgs, const double *, double *, double *, int32_t *, int);

// Whether a step in variant v sweeps its subgrids without species in the
// paired body: the default options, parts of at least two planes, and a batch
// not known to hold none (the instance with both bodies runs the 11-field
// body about 1 % slower than the 11-field instance: one allocation of
// registers serves both bodies).
bool pairs(const StepArgs &a, int v) {
    return !a.unpaired && !a.vel && !a.steepen && !a.flatten && kVariants[v].log_parts < 3;
}

template <bool GATHER>
FusedKernel fused_kernel_g(const StepArgs &a, int v) {
    const bool cw = a.steepen || a.flatten;
    if (a.vel) return cw ? k_fused<true, true, GATHER> : k_fused<true, false, GATHER>;
    if (cw) return k_fused<false, true, GATHER>;
    return pairs(a, v) ? k_fused<false, false, GATHER, true> : k_fused<false, false, GATHER>;
}

FusedKernel fused_kernel(const StepArgs &a, int v) {
    return a.gsrc ? fused_kernel_g<true>(a, v) : fused_kernel_g<false>(a, v);
}

dim3 grid_of(const StepArgs &a, int v) {
    const Variant &V = kVariants[v];
    const int items = a.n_sub << V.log_parts;
    int g = V.grid_per_cu ? V.grid_per_cu * device_cus() : items;
    if (g > items) g = items;
    return dim3(g < 1 ? 1 : g);
}

}  // namespace

int fused_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const char *fused_variant_name(int v) {
    return (v >= 0 && v < fused_variant_count()) ? kVariants[v].name : "?";
}
int fused_variant_order(int v) {
    return (v >= 0 && v < fused_variant_count()) ? kVariants[v].order : 0;
}
bool fused_needs_scratch(const StepArgs &, int v) {
    return v >= 0 && v < fused_variant_count() && (kVariants[v].log_parts > 0 || kVariants[v].dyn);
}
int64_t fused_scratch_bytes(int n_sub) { return fused_scratch_bytes_for(n_sub > 0 ? n_sub : 0); }

int fused_default_variant(int n_sub) {
    // The launch of fewest rounds of work items, each round costing one
    // part's time: ceil(n_sub P / CUs) t(P), with t(P) the time of one part
    // relative to a whole sweep as measured on an MI355X (141.5, 82.9, 52.2
    // and 36.4 us for P = 1, 2, 4, 8).  P = 1 launches as persistent-2x (the
    // second wave of workgroups evens out the tail).
    static const double kPartCost[4] = {1.0, 0.586, 0.369, 0.257};
    const int64_t cus = device_cus();
    int best = 0;
    double best_t = 0.0;
    for (int lp = 0; lp <= 3; lp++) {
        const int64_t items = (int64_t)n_sub << lp;
        const double t = (double)((items + cus - 1) / cus) * kPartCost[lp];
        if (lp == 0 || t < best_t * 0.98) {
            best = lp;
            best_t = t;
        }
    }
    return best == 0 ? 1 : kVariantSplit2 + best - 1;
}

void apply_variant(StepArgs &a, int v) {
    a.log_parts = kVariants[v].log_parts;
    a.dyn = kVariants[v].dyn;
}

hipError_t launch_fused_step(const StepArgs &a0, const double *U_in, double *U_out,
                             double *amax, int32_t *status, int variant, hipStream_t st) {
    if (a0.n_sub == 0) return hipSuccess;
    // the ghost map addresses NB-pitched blocks
    if (GNB != NB && a0.gsrc) return hipErrorInvalidValue;
    StepArgs a = a0;
    apply_variant(a, variant);
    if (fused_needs_scratch(a, variant) && !a.scratch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fused_kernel(a, variant), grid_of(a, variant), dim3(NT), 0, st,
                       fused_args(a), U_in, U_out, amax, status, kVariants[variant].order);
    return hipGetLastError();
}

int fused_global_pitch() { return GNB; }

}  // namespace hydro
