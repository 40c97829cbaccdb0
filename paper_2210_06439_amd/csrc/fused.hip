// fused.hip -- the fused hydro stage: PPM reconstruction, central-upwind
// flux with Simpson quadrature and the finite-volume update in one persistent
// launch, with no intermediate array in HBM.
//
// Mapping (one workgroup of 4 waves per subgrid, looping over subgrids):
//   * The subgrid is swept plane by plane along z.  LDS holds a rolling
//     window of 5 z-planes of every field (planes k-2..k+2 around the current
//     plane k); the next plane is prefetched into registers one step ahead.
//   * Waves 0, 1, 2 own the x-, y- and z-faces of the 8x8 interior cells of
//     plane k (lane = cell).  The 13 PPM lines of a cell are split between
//     the three waves (4, 4 and 5 lines; every line is computed once); each
//     line yields the reconstructed state at two opposite surface points,
//     which go through LDS to every wave whose faces contain them.
//   * Wave 3 handles the 32 "ring" cells just outside the interior in x and
//     y (2 lanes each); they need only the 9 points of the one face they
//     share with the interior.
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
namespace {

constexpr int NT = 256;
constexpr int SLOTS = 5;               // window planes
constexpr int PT = 16;                 // doubles per exchanged point
constexpr int PV = 11;                 // point slots: V[0..10], then
constexpr int P_VX = 11, P_P = 14, P_CS = 15;   // vx vy vz, p, cs
constexpr int NACC = 24;               // doubles per face-side partial

// LDS layout, in doubles
constexpr int WIN_D = SLOTS * NF_MAX * NPLANE;       // 10780
constexpr int XCH_D = 3 * 2 * PT * 64;               // 6144
constexpr int ZL_D = NACC * 64;                      // 1536
constexpr int KEEP_D = 2 * NF_MAX * 64;              // 1408
constexpr int LDS_D = WIN_D + XCH_D + ZL_D + KEEP_D + 8;
static_assert(LDS_D * 8 + 32 <= 163840, "LDS budget");

// combine-phase sub-regions of XCH
constexpr int XR_OFF = 0;                            // [24][2][8][9]
constexpr int XF_OFF = NACC * 2 * 8 * 9;             // [11][2][8][9]
constexpr int DX_OFF = 0;                            // [2][11][64] (aliases XR)
static_assert(XF_OFF + NF_MAX * 2 * 8 * 9 <= XCH_D, "combine layout");

// Accumulator layout inside NACC: sv[0..10], sf[1..10] at 11..20, sp, lp, lm.
struct Acc {
    double sv[NF_MAX];
    double sf[NF_MAX];   // sf[0] unused: the density flux is S_V of the normal momentum
    double sp;           // sum w p (added to the normal momentum's flux)
    double lp, lm;       // max(u_n + c), min(u_n - c)
};

__device__ __forceinline__ void acc_zero(Acc &a) {
#pragma unroll
    for (int f = 0; f < NF_MAX; f++) {
        a.sv[f] = 0.0;
        a.sf[f] = 0.0;
    }
    a.sp = 0.0;
    a.lp = -INFINITY;
    a.lm = INFINITY;
}

// ---- the 13 lines: n = 14 + L, (dx,dy,dz) from the base-3 digits of n -------

__device__ __host__ constexpr int ldx(int L) { return (14 + L) % 3 - 1; }
__device__ __host__ constexpr int ldy(int L) { return ((14 + L) / 3) % 3 - 1; }
__device__ __host__ constexpr int ldz(int L) { return (14 + L) / 9 - 1; }

// Lines produced by wave w in round r (-1: idle).  Every line's support
// contains its producer's axis; x: X, (1,1,0), (1,0,1), (1,1,1);
// y: Y, (-1,1,0), (0,1,1), (-1,1,1); z: Z, (-1,0,1), (0,-1,1), (1,-1,1), (-1,-1,1).
__device__ __host__ constexpr int line_of(int w, int r) {
    return w == 0 ? (r == 0 ? 0 : r == 1 ? 3 : r == 2 ? 9 : r == 3 ? 12 : -1)
         : w == 1 ? (r == 0 ? 2 : r == 1 ? 1 : r == 2 ? 11 : r == 3 ? 10 : -1)
                  : (r == 0 ? 8 : r == 1 ? 7 : r == 2 ? 5 : r == 3 ? 6 : 4);
}

__device__ __forceinline__ int comp(int L, int axis) {
    return axis == 0 ? ldx(L) : axis == 1 ? ldy(L) : ldz(L);
}

// Simpson weight of a surface point from its two tangential offsets.
__device__ __forceinline__ double simpson_w(int t1, int t2) {
    const double w1a = t1 == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
    const double w1b = t2 == 0 ? 4.0 / 6.0 : 1.0 / 6.0;
    return w1a * w1b;
}

// ---- PPM in branch-free form ---------------------------------------------

// x with its sign bit flipped where s (a high-word mask) has it set.
__device__ __forceinline__ double flip(double x, int s) {
    return __hiloint2double(__double2hiint(x) ^ s, __double2loint(x));
}

// Monotonised-central slope from the two one-sided differences.
__device__ __forceinline__ double mc_slope(double dm, double dp) {
    double d = 0.5 * (dm + dp);
    int s = __double2hiint(d) & (int)0x80000000;
    double t = fmin(flip(dm, s), flip(dp, s));       // both > 0 iff same sign as d
    t = fmax(fmin(fabs(d), 2.0 * t), 0.0);
    return flip(t, s);
}

// PPM on u_{-2..2}: the Colella-Woodward monotonicity step written in its
// equivalent clamp form (a = q+ - u0, b = u0 - q-: flatten if a b <= 0, else
// |b| <= 2|a| and |a| <= 2|b|), which needs no division and no branches.
__device__ __forceinline__ void ppm_fast(double um2, double um1, double u0, double up1, double up2,
                                double &qp, double &qm) {
    const double sixth = 1.0 / 6.0;
    double sm = mc_slope(um1 - um2, u0 - um1);
    double s0 = mc_slope(u0 - um1, up1 - u0);
    double sp = mc_slope(up1 - u0, up2 - up1);
    double ip = fma(s0 - sp, sixth, 0.5 * (u0 + up1));
    double im = fma(sm - s0, sixth, 0.5 * (um1 + u0));
    double a = ip - u0, b = u0 - im;
    int s = __double2hiint(a) & (int)0x80000000;
    double aa = fabs(a);
    double sb = flip(b, s);                             // |b| if b has a's sign
    double bn = fmax(fmin(sb, 2.0 * aa), 0.0);
    double an = fmax(fmin(aa, 2.0 * sb), 0.0);
    qp = u0 + flip(an, s);
    qm = u0 - flip(bn, s);
}

// ---- point state ----------------------------------------------------------

struct PState {
    double vx, vy, vz, p, cs;
};

__device__ __forceinline__ PState pstate(double rho, double sx, double sy, double sz, double E,
                                double tau, double gamma, double gm1, double de, int &bits) {
    PState st;
    double r = 1.0 / rho;
    st.vx = sx * r;
    st.vy = sy * r;
    st.vz = sz * r;
    double ek = 0.5 * fma(sz, st.vz, fma(sy, st.vy, sx * st.vx));
    double ei = E - ek;
    if (ei < de * E) ei = pow(tau, gamma);
    st.p = gm1 * ei;
    st.cs = sqrt((gamma * st.p) * r);
    bits |= (rho <= 0.0 ? HYDRO_STATUS_RHO : 0) | (st.p <= 0.0 ? HYDRO_STATUS_P : 0);
    return st;
}

__device__ __forceinline__ void acc_hydro(Acc &a, const double *V, double un, double p, double cs,
                                 double w) {
    double wun = w * un;
#pragma unroll
    for (int f = 0; f < 6; f++) a.sv[f] = fma(w, V[f], a.sv[f]);
    a.sf[1] = fma(wun, V[1], a.sf[1]);
    a.sf[2] = fma(wun, V[2], a.sf[2]);
    a.sf[3] = fma(wun, V[3], a.sf[3]);
    a.sf[4] = fma(wun, V[4] + p, a.sf[4]);
    a.sf[5] = fma(wun, V[5], a.sf[5]);
    a.sp = fma(w, p, a.sp);
    a.lp = fmax(a.lp, un + cs);
    a.lm = fmin(a.lm, un - cs);
}

__device__ __forceinline__ void acc_species(Acc &a, int f, double v, double w, double wun) {
    a.sv[f] = fma(w, v, a.sv[f]);
    a.sf[f] = fma(wun, v, a.sf[f]);
}

// ---- LDS helpers ------------------------------------------------------------

__device__ __forceinline__ const double *win_field(const double *win, int plane, int f) {
    return win + ((plane % SLOTS) * NF_MAX + f) * NPLANE;
}

// The five window offsets of the line through (i,j,k) along (dx,dy,dz).
struct Line5 {
    int o[5];
};

__device__ __forceinline__ Line5 line5(int i, int j, int k, int dx, int dy, int dz) {
    Line5 l;
#pragma unroll
    for (int m = -2; m <= 2; m++) {
        int pl = (k + m * dz) % SLOTS;
        l.o[m + 2] = pl * NF_MAX * NPLANE + (j + m * dy) * NB + (i + m * dx);
    }
    return l;
}

__device__ __forceinline__ void ppm_at(const double *win, const Line5 &l, int f, double &qp, double &qm) {
    const int fo = f * NPLANE;
    ppm_fast(win[l.o[0] + fo], win[l.o[1] + fo], win[l.o[2] + fo], win[l.o[3] + fo],
             win[l.o[4] + fo], qp, qm);
}

// Store/load of a 24-double partial at stride `st` (component-major layouts).
__device__ __forceinline__ void acc_store(double *base, int st, const Acc &a, int nf) {
#pragma unroll
    for (int f = 0; f < NF_MAX; f++)
        if (f < nf) base[f * st] = a.sv[f];
#pragma unroll
    for (int f = 1; f < NF_MAX; f++)
        if (f < nf) base[(10 + f) * st] = a.sf[f];
    base[21 * st] = a.sp;
    base[22 * st] = a.lp;
    base[23 * st] = a.lm;
}

// Face flux from the left partial L and a right partial stored at (R, st)
// (or the reverse when `left_in_lds`), normal axis `axis`.  Writes Fb[f] for
// f < nf and returns max(a+, -a-).
__device__ __forceinline__ double combine(const Acc &mine, const double *other, int st, bool mine_is_left,
                                 int axis, int nf, double *Fb) {
    const double lp = fmax(mine.lp, other[22 * st]);
    const double lm = fmin(mine.lm, other[23 * st]);
    const double ap = fmax(0.0, lp);
    const double am = fmin(0.0, lm);
    const double inv = 1.0 / (ap - am);
    const double apam = ap * am;
    // left/right selectors
    const double cl = mine_is_left ? ap : -am;       // coefficient of my S_F
    const double co = mine_is_left ? -am : ap;       // coefficient of the other S_F
    const double sg = mine_is_left ? 1.0 : -1.0;     // (S_V^R - S_V^L) = sg * (other - mine)
    const double osp = other[21 * st];
    // (value selects, not an lvalue conditional: the latter would index the
    // accumulator through a pointer and force it out of registers)
    const double m1 = mine.sv[1], m2 = mine.sv[2], m3 = mine.sv[3];
    const double ms_axis = axis == 0 ? m1 : (axis == 1 ? m2 : m3);
    const double os_axis = other[(1 + axis) * st];
#pragma unroll
    for (int f = 0; f < NF_MAX; f++) {
        if (f < nf) {
            double sfm, sfo;
            if (f == 0) {
                sfm = ms_axis;
                sfo = os_axis;
            } else {
                sfm = mine.sf[f];
                sfo = other[(10 + f) * st];
                if (f == 1 + axis) {
                    sfm += mine.sp;
                    sfo += osp;
                }
            }
            double dv = sg * (other[f * st] - mine.sv[f]);
            Fb[f] = fma(cl, sfm, co * sfo) * inv + (apam * dv) * inv;
        }
    }
    return fmax(ap, -am);
}

// ---- the kernel ---------------------------------------------------------------

__global__ __launch_bounds__(NT, 1) void k_fused(StepArgs a, const double *__restrict__ U,
                                                 double *__restrict__ Uo,
                                                 double *__restrict__ amax,
                                                 int32_t *__restrict__ status, int order) {
    __shared__ double lds[LDS_D];
    __shared__ int red_bits[4];
    double *win = lds;
    double *xch = lds + WIN_D;
    double *zl = xch + XCH_D;
    double *keep = zl + ZL_D;          // [0: F_z of the previous face][1: dFx+dFy][11][64]
    double *red = keep + KEEP_D;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ci = 3 + (lane & 7), cj = 3 + (lane >> 3);
    // ring cell of wave 3 (two lanes per cell)
    const int rc = lane >> 1, half = lane & 1;
    const int r_axis = rc >> 4;
    const int r_side = (rc >> 3) & 1;        // 0: low side (left cell), 1: high side
    const int r_pos = 3 + (rc & 7);
    const int ri = r_axis == 0 ? (r_side ? 11 : 2) : r_pos;
    const int rj = r_axis == 0 ? r_pos : (r_side ? 11 : 2);

    const double gamma = a.gamma, gm1 = a.gamma - 1.0, de = a.de_switch;

    for (int it = blockIdx.x; it < a.n_sub; it += gridDim.x) {
        const int s = order ? (a.n_sub - 1 - it) : it;
        const int ns = a.n_species[s];
        const int64_t off = a.offset[s];
        if (ns < 0 || ns > 5 || off < 0 || (off & 1)) {
            if (tid == 0) {
                amax[s] = 0.0;
                if (status) status[s] = HYDRO_STATUS_BADMETA;
            }
            continue;
        }
        const int nf = 6 + ns;
        const double lam = a.dt / a.h[s];
        const double *Us = U + off;
        double *Os = Uo + off;
        const int64_t fst = a.fstride;
        double amax_l = 0.0;
        int bits = 0;

        __syncthreads();   // previous subgrid's LDS reads are done
        // window: planes 0..4
        for (int pl = 0; pl < SLOTS; pl++)
            for (int e = tid; e < nf * NPLANE; e += NT) {
                int f = e / NPLANE, c = e - f * NPLANE;
                win[(pl * NF_MAX + f) * NPLANE + c] = Us[f * fst + pl * NPLANE + c];
            }
        double pf[9];
#pragma unroll
        for (int q = 0; q < 9; q++) {   // prefetch plane 5
            int e = tid + q * NT;
            pf[q] = 0.0;
            if (e < nf * NPLANE) {
                int f = e / NPLANE, c = e - f * NPLANE;
                pf[q] = Us[f * fst + 5 * NPLANE + c];
            }
        }
        __syncthreads();

        Acc A, B;
        for (int k = 2; k <= 11; k++) {
            if (k >= 3) {
                // plane k+2 from the prefetch registers, then prefetch k+3
#pragma unroll
                for (int q = 0; q < 9; q++) {
                    int e = tid + q * NT;
                    if (e < nf * NPLANE) {
                        int f = e / NPLANE, c = e - f * NPLANE;
                        win[(((k + 2) % SLOTS) * NF_MAX + f) * NPLANE + c] = pf[q];
                    }
                }
                if (k + 3 <= 13) {
#pragma unroll
                    for (int q = 0; q < 9; q++) {
                        int e = tid + q * NT;
                        if (e < nf * NPLANE) {
                            int f = e / NPLANE, c = e - f * NPLANE;
                            pf[q] = Us[f * fst + (k + 3) * NPLANE + c];
                        }
                    }
                }
                __syncthreads();
            }
            acc_zero(A);
            acc_zero(B);

            if (k == 2 || k == 11) {
                // ---- z face layer: 9 points of one side of the boundary z-faces
                const int dzs = k == 2 ? 1 : -1;
                for (int r = 0; r < 3; r++) {
                    const int t = wave + 4 * r;
                    if (t < 9) {
                        const int tx = t % 3 - 1, ty = t / 3 - 1;
                        Line5 l = line5(ci, cj, k, tx, ty, dzs);
                        double *pt = xch + wave * PT * 64 + lane;
                        double q[6], qm;
#pragma unroll
                        for (int f = 0; f < 6; f++) ppm_at(win, l, f, q[f], qm);
                        PState st = pstate(q[0], q[1], q[2], q[3], q[4], q[5], gamma, gm1, de, bits);
#pragma unroll
                        for (int f = 0; f < 6; f++) pt[f * 64] = q[f];
#pragma unroll
                        for (int f = 6; f < NF_MAX; f++)
                            if (f < nf) {
                                double v;
                                ppm_at(win, l, f, v, qm);
                                pt[f * 64] = v;
                            }
                        pt[(P_VX + 2) * 64] = st.vz;
                        pt[P_P * 64] = st.p;
                        pt[P_CS * 64] = st.cs;
                    }
                    __syncthreads();
                    if (wave == 2) {
                        for (int w = 0; w < 4; w++) {
                            const int t2 = w + 4 * r;
                            if (t2 >= 9) break;
                            const double wt = simpson_w(t2 % 3 - 1, t2 / 3 - 1);
                            const double *pt = xch + w * PT * 64 + lane;
                            double V[6];
#pragma unroll
                            for (int f = 0; f < 6; f++) V[f] = pt[f * 64];
                            const double un = pt[(P_VX + 2) * 64];
                            // A holds this side of the boundary face in both layers
                            acc_hydro(A, V, un, pt[P_P * 64], pt[P_CS * 64], wt);
                            const double wun = wt * un;
#pragma unroll
                            for (int f = 6; f < NF_MAX; f++)
                                if (f < nf) acc_species(A, f, pt[f * 64], wt, wun);
                        }
                    }
                    __syncthreads();
                }
                if (wave == 2) {
                    if (k == 2) {
                        acc_store(zl + lane, 64, A, nf);
                    } else {
                        // face (10|11): left partial from the previous step, right = A
                        double Fb[NF_MAX];
                        double af = combine(A, zl + lane, 64, false, 2, nf, Fb);
                        amax_l = fmax(amax_l, af);
                        const int cidx = (k - 1) * NPLANE + cj * NB + ci;
#pragma unroll
                        for (int f = 0; f < NF_MAX; f++)
                            if (f < nf) {
                                double dfz = Fb[f] - keep[f * 64 + lane];
                                double sxy = keep[(NF_MAX + f) * 64 + lane];
                                double u = win_field(win, k - 1, f)[cj * NB + ci];
                                double v = u - lam * (sxy + dfz);
                                if (!isfinite(v) || !isfinite(Fb[f])) bits |= HYDRO_STATUS_NONFINITE;
                                Os[f * fst + cidx] = v;
                            }
                    }
                }
                continue;
            }

            // ---- interior plane: 5 rounds of line production and consumption
#pragma unroll
            for (int r = 0; r < 5; r++) {
                if (wave < 3) {
                    const int L = line_of(wave, r);
                    if (L >= 0) {
                        Line5 l = line5(ci, cj, k, ldx(L), ldy(L), ldz(L));
                        double qp[6], qm[6];
#pragma unroll
                        for (int f = 0; f < 6; f++) ppm_at(win, l, f, qp[f], qm[f]);
                        PState sp = pstate(qp[0], qp[1], qp[2], qp[3], qp[4], qp[5], gamma, gm1, de, bits);
                        PState sm = pstate(qm[0], qm[1], qm[2], qm[3], qm[4], qm[5], gamma, gm1, de, bits);
                        double *pp = xch + (wave * 2 + 0) * PT * 64 + lane;
                        double *pm = xch + (wave * 2 + 1) * PT * 64 + lane;
#pragma unroll
                        for (int f = 0; f < 6; f++) {
                            pp[f * 64] = qp[f];
                            pm[f * 64] = qm[f];
                        }
                        pp[P_VX * 64] = sp.vx; pp[(P_VX + 1) * 64] = sp.vy; pp[(P_VX + 2) * 64] = sp.vz;
                        pp[P_P * 64] = sp.p; pp[P_CS * 64] = sp.cs;
                        pm[P_VX * 64] = sm.vx; pm[(P_VX + 1) * 64] = sm.vy; pm[(P_VX + 2) * 64] = sm.vz;
                        pm[P_P * 64] = sm.p; pm[P_CS * 64] = sm.cs;
#pragma unroll
                        for (int f = 6; f < NF_MAX; f++)
                            if (f < nf) {
                                double vp, vm;
                                ppm_at(win, l, f, vp, vm);
                                pp[f * 64] = vp;
                                pm[f * 64] = vm;
                            }
                    }
                } else {
                    const int t = half ? 5 + r : r;
                    if (t < 9) {
                        const int t1 = t % 3 - 1, t2 = t / 3 - 1;
                        const int dn = r_side ? -1 : 1;    // normal component
                        const int Dx = r_axis == 0 ? dn : t1;
                        const int Dy = r_axis == 0 ? t1 : dn;
                        Line5 l = line5(ri, rj, k, Dx, Dy, t2);
                        double q[6], qm;
#pragma unroll
                        for (int f = 0; f < 6; f++) ppm_at(win, l, f, q[f], qm);
                        PState st = pstate(q[0], q[1], q[2], q[3], q[4], q[5], gamma, gm1, de, bits);
                        const double wt = simpson_w(t1, t2);
                        const double vx = st.vx, vy = st.vy;
                        const double un = r_axis == 0 ? vx : vy;
                        acc_hydro(A, q, un, st.p, st.cs, wt);
                        const double wun = wt * un;
#pragma unroll
                        for (int f = 6; f < NF_MAX; f++)
                            if (f < nf) {
                                double v;
                                ppm_at(win, l, f, v, qm);
                                acc_species(A, f, v, wt, wun);
                            }
                    }
                }
                __syncthreads();
                if (wave < 3) {
                    const int ax = wave;
                    const int b1 = ax == 0 ? 1 : 0, b2 = ax == 2 ? 1 : 2;
#pragma unroll
                    for (int p = 0; p < 3; p++) {
                        const int L = line_of(p, r);
                        if (L < 0) continue;
                        const int dA = comp(L, ax);
                        if (dA == 0) continue;
#pragma unroll
                        for (int pm = 0; pm < 2; pm++) {
                            const int sgn = pm == 0 ? 1 : -1;
                            const int t1 = sgn * comp(L, b1), t2 = sgn * comp(L, b2);
                            const double wt = simpson_w(t1, t2);
                            const double *pt = xch + (p * 2 + pm) * PT * 64 + lane;
                            double V[6];
#pragma unroll
                            for (int f = 0; f < 6; f++) V[f] = pt[f * 64];
                            const double un = pt[(P_VX + ax) * 64];
                            const double pr = pt[P_P * 64], cs = pt[P_CS * 64];
                            const double wun = wt * un;
                            if (sgn * dA > 0) {
                                acc_hydro(A, V, un, pr, cs, wt);
#pragma unroll
                                for (int f = 6; f < NF_MAX; f++)
                                    if (f < nf) acc_species(A, f, pt[f * 64], wt, wun);
                            } else {
                                acc_hydro(B, V, un, pr, cs, wt);
#pragma unroll
                                for (int f = 6; f < NF_MAX; f++)
                                    if (f < nf) acc_species(B, f, pt[f * 64], wt, wun);
                            }
                        }
                    }
                }
                __syncthreads();
            }

            // ---- face fluxes of plane k and the update of plane k-1
            if (wave == 3) {
                // the two lanes of a ring cell hold partial sums: add them
#pragma unroll
                for (int f = 0; f < NF_MAX; f++) {
                    A.sv[f] += __shfl_xor(A.sv[f], 1);
                    A.sf[f] += __shfl_xor(A.sf[f], 1);
                }
                A.sp += __shfl_xor(A.sp, 1);
                A.lp = fmax(A.lp, __shfl_xor(A.lp, 1));
                A.lm = fmin(A.lm, __shfl_xor(A.lm, 1));
            }
            // right-side partials of the x and y faces -> LDS  ([24][2][8][9])
            constexpr int RST = 2 * 8 * 9;
            if (wave == 0) acc_store(xch + XR_OFF + (0 * 8 + (cj - 3)) * 9 + (ci - 3), RST, B, nf);
            if (wave == 1) acc_store(xch + XR_OFF + (1 * 8 + (ci - 3)) * 9 + (cj - 3), RST, B, nf);
            if (wave == 3 && half == 0 && r_side == 1)
                acc_store(xch + XR_OFF + (r_axis * 8 + (r_pos - 3)) * 9 + 8, RST, A, nf);
            __syncthreads();
            // left owners form the face fluxes ([11][2][8][9])
            double Fb[NF_MAX];
            if (wave < 2 || (wave == 3 && half == 0 && r_side == 0)) {
                const int ax = wave < 2 ? wave : r_axis;
                const int row = wave == 0 ? cj - 3 : wave == 1 ? ci - 3 : r_pos - 3;
                const int p = wave == 0 ? ci - 2 : wave == 1 ? cj - 2 : 0;
                const double *R = xch + XR_OFF + (ax * 8 + row) * 9 + p;
                double af = combine(A, R, RST, true, ax, nf, Fb);
                amax_l = fmax(amax_l, af);
                double *Fo = xch + XF_OFF + (ax * 8 + row) * 9 + p;
#pragma unroll
                for (int f = 0; f < NF_MAX; f++)
                    if (f < nf) {
                        Fo[f * RST] = Fb[f];
                        if (!isfinite(Fb[f])) bits |= HYDRO_STATUS_NONFINITE;
                    }
            }
            if (wave == 2) {
                // z-face (k-1|k): left partial from the previous step, right = B
                double Fz[NF_MAX];
                double af = combine(B, zl + lane, 64, false, 2, nf, Fz);
                amax_l = fmax(amax_l, af);
                const int cidx = (k - 1) * NPLANE + cj * NB + ci;
#pragma unroll
                for (int f = 0; f < NF_MAX; f++)
                    if (f < nf) {
                        if (k >= 4) {
                            double dfz = Fz[f] - keep[f * 64 + lane];
                            double sxy = keep[(NF_MAX + f) * 64 + lane];
                            double u = win_field(win, k - 1, f)[cj * NB + ci];
                            double v = u - lam * (sxy + dfz);
                            if (!isfinite(v)) bits |= HYDRO_STATUS_NONFINITE;
                            Os[f * fst + cidx] = v;
                        }
                        if (!isfinite(Fz[f])) bits |= HYDRO_STATUS_NONFINITE;
                        keep[f * 64 + lane] = Fz[f];
                    }
                acc_store(zl + lane, 64, A, nf);
            }
            __syncthreads();
            // x/y owners: flux differences of their cells -> LDS ([2][11][64])
            if (wave < 2) {
                const int ax = wave;
                const int row = wave == 0 ? cj - 3 : ci - 3;
                const int p = wave == 0 ? ci - 3 : cj - 3;      // left face of the cell
                const double *Fl = xch + XF_OFF + (ax * 8 + row) * 9 + p;
                double *d = xch + DX_OFF + ax * NF_MAX * 64 + lane;
#pragma unroll
                for (int f = 0; f < NF_MAX; f++)
                    if (f < nf) d[f * 64] = Fb[f] - Fl[f * RST];
            }
            __syncthreads();
            if (wave == 2) {
#pragma unroll
                for (int f = 0; f < NF_MAX; f++)
                    if (f < nf)
                        keep[(NF_MAX + f) * 64 + lane] =
                            xch[DX_OFF + f * 64 + lane] + xch[DX_OFF + (NF_MAX + f) * 64 + lane];
            }
            // (the next step's window barrier orders these reads before XCH reuse)
        }

        // ---- per-subgrid speed and status
        for (int o = 32; o > 0; o >>= 1) {
            amax_l = fmax(amax_l, __shfl_xor(amax_l, o));
            bits |= __shfl_xor(bits, o);
        }
        if (lane == 0) {
            red[wave] = amax_l;
            red_bits[wave] = bits;
        }
        __syncthreads();
        if (tid == 0) {
            double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            int b = red_bits[0] | red_bits[1] | red_bits[2] | red_bits[3];
            if (!isfinite(m)) b |= HYDRO_STATUS_NONFINITE;
            amax[s] = m;
            if (status) status[s] = b;
        }
    }
}

struct Variant {
    const char *name;
    int grid_per_cu;   // persistent workgroups per CU; 0 = one workgroup per subgrid
    int order;         // 0: subgrid order, 1: reverse order
};

constexpr Variant kVariants[] = {
    {"persistent-1x", 1, 0},
    {"persistent-2x", 2, 0},
    {"one-per-subgrid", 0, 0},
    {"persistent-1x-rev", 1, 1},
};

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

dim3 grid_of(const StepArgs &a, int v) {
    const Variant &V = kVariants[v];
    int g = V.grid_per_cu ? V.grid_per_cu * device_cus() : a.n_sub;
    if (g > a.n_sub) g = a.n_sub;
    return dim3(g < 1 ? 1 : g);
}

}  // namespace

int fused_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const char *fused_variant_name(int v) {
    return (v >= 0 && v < fused_variant_count()) ? kVariants[v].name : "?";
}

hipError_t launch_fused_step(const StepArgs &a, const double *U_in, double *U_out,
                             double *amax, int32_t *status, int variant, hipStream_t st) {
    if (a.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fused, grid_of(a, variant), dim3(NT), 0, st, a, U_in, U_out, amax,
                       status, kVariants[variant].order);
    return hipGetLastError();
}

hipError_t fused_kernel_node_params(const StepArgs &a, const double *U_in, double *U_out,
                                    double *amax, int32_t *status, int variant,
                                    hipKernelNodeParams *out, void **args) {
    // args must point at storage for the kernel's arguments, filled by the caller
    out->func = reinterpret_cast<void *>(k_fused);
    out->gridDim = grid_of(a, variant);
    out->blockDim = dim3(NT);
    out->sharedMemBytes = 0;
    out->kernelParams = args;
    out->extra = nullptr;
    (void)U_in; (void)U_out; (void)amax; (void)status;
    return hipSuccess;
}

}  // namespace hydro
