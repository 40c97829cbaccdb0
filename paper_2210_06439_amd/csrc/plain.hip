// plain.hip -- the unfused stages: reconstruct, flux, divergence.
//
// These kernels write the full intermediate arrays Q (26 quadrature values
// per cell and field) and F (averaged face fluxes) to memory, one stage per
// launch, the way the paper's `reconstruct` and `flux` kernels each run per
// subgrid (Sec. III-D).  Every floating-point expression is evaluated in the
// order the method's definition states (contraction off), so the results are
// reproducible bit for bit across launch shapes.
#include "hydro_internal.hpp"

#pragma clang fp contract(off)

namespace hydro {
namespace {

// ---- geometry --------------------------------------------------------------

// The 13 lines are the directions n = 9(dz+1) + 3(dy+1) + (dx+1) in 14..26;
// their storage slot is n-1, the opposite direction's slot is 26-n.
__device__ inline void line_dir(int line, int &dx, int &dy, int &dz) {
    int n = 14 + line;
    dz = n / 9 - 1;
    dy = (n / 3) % 3 - 1;
    dx = n % 3 - 1;
}

__device__ inline int dir_slot(int dx, int dy, int dz) {
    int n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
    return n < 13 ? n : n - 1;
}

__device__ inline int qcell(int i, int j, int k) {   // cell in [2, NB-2)^3 -> 0..QCELL-1
    return ((k - 2) * QN + (j - 2)) * QN + (i - 2);
}

// Face index of the face whose left cell is (i,j,k) on `axis`: the faces of
// an axis form a box of extent N+1 along it and N across, x fastest.
__device__ inline int face_idx(int axis, int i, int j, int k) {
    constexpr int n = NSUB;
    if (axis == 0) return ((k - NG) * n + (j - NG)) * (n + 1) + (i - 2);
    if (axis == 1) return ((k - NG) * (n + 1) + (j - 2)) * n + (i - NG);
    return ((k - 2) * n + (j - NG)) * n + (i - NG);
}

__device__ inline bool meta_ok(const StepArgs &a, int s, int &nf, int64_t &off) {
    int ns = a.n_species[s];
    off = a.offset[s];
    nf = 6 + ns;
    return ns >= 0 && ns <= 5 && off >= 0;
}

// ---- PPM (Colella-Woodward 1984, MC slopes) ----------------------------------

__device__ inline double mc_slope(double ul, double uc, double ur) {
    double dm = uc - ul;
    double dp = ur - uc;
    double d = 0.5 * (dp + dm);
    if (dp * dm > 0.0) {
        double lim = fmin(2.0 * fabs(dm), 2.0 * fabs(dp));
        return copysign(fmin(fabs(d), lim), d);
    }
    return 0.0;
}

__device__ inline void ppm(double um2, double um1, double u0, double up1, double up2,
                           double &qp, double &qm) {
    const double sixth = 1.0 / 6.0;
    double s_m = mc_slope(um2, um1, u0);
    double s_0 = mc_slope(um1, u0, up1);
    double s_p = mc_slope(u0, up1, up2);
    qp = 0.5 * (u0 + up1) - (s_p - s_0) * sixth;
    qm = 0.5 * (um1 + u0) - (s_0 - s_m) * sixth;
    if ((qp - u0) * (u0 - qm) <= 0.0) {
        qp = u0;
        qm = u0;
    } else {
        double dq = qp - qm;
        double m6 = 6.0 * (u0 - 0.5 * (qm + qp));
        if (dq * m6 > dq * dq) {
            qm = 3.0 * u0 - 2.0 * qp;
        } else if (-(dq * dq) > dq * m6) {
            qp = 3.0 * u0 - 2.0 * qm;
        }
    }
}

// ---- Colella-Woodward (1984) refinements of the interface values ------------
// Contact steepening (density) and flattening (all fields), applied to the
// fourth-order interface values before the monotonicity constraint.  They
// need the pressures of the five cells of the line (ideal gas with the
// dual-energy switch, the point-state formulas) and the velocities along the
// line direction.

// Pressure and velocity along (dx, dy, dz) of cell c of a subgrid.
__device__ inline void cell_p_un(const StepArgs &a, const double *Us, int c, int dx, int dy,
                                 int dz, double &p, double &un) {
    const int64_t fs = a.fstride;
    const double rho = Us[c];
    const double sx = Us[fs + c], sy = Us[2 * fs + c], sz = Us[3 * fs + c];
    const double r = 1.0 / rho;
    const double vx = sx * r, vy = sy * r, vz = sz * r;
    const double ek = 0.5 * ((sx * vx + sy * vy) + sz * vz);
    const double E = Us[4 * fs + c];
    double ei = E - ek;
    if (ei < a.de_switch * E) ei = pow(Us[5 * fs + c], a.gamma);
    p = (a.gamma - 1.0) * ei;
    un = (dx * vx + dy * vy) + dz * vz;
}

// Steepening weight of the middle cell: a contact (opposite second
// differences of the density on the two sides, a density jump above eps1 of
// the smaller density and at least the relative pressure jump / (gamma K0)),
// then eta = clamp(eta1 (eta~ - eta2), 0, 1) with
// eta~ = -(D_{j+1} - D_{j-1}) / (6 (rho_{j+1} - rho_{j-1})).
__device__ inline double steepen_weight(double gamma, const double *rho, const double *p) {
    // outer pair first: the reversed line gives the same bits
    const double d2m = (rho[0] + rho[2]) - 2.0 * rho[1];
    const double d2p = (rho[2] + rho[4]) - 2.0 * rho[3];
    const double drho = rho[3] - rho[1];
    if (!(d2p * d2m < 0.0)) return 0.0;
    if (!(fabs(drho) - CW_EPS1 * fmin(fabs(rho[3]), fabs(rho[1])) > 0.0)) return 0.0;
    const double jump_rho = gamma * CW_K0 * fabs(drho) / fmin(rho[3], rho[1]);
    const double jump_p = fabs(p[3] - p[1]) / fmin(p[3], p[1]);
    if (!(jump_rho >= jump_p)) return 0.0;
    const double et = -(d2p - d2m) / (6.0 * drho);
    return fmax(0.0, fmin(CW_ETA1 * (et - CW_ETA2), 1.0));
}

// Flattening weight of the middle cell: in a compression along the line with
// a relative pressure jump above eps,
// clamp(omega2 ((p_{j+1} - p_{j-1}) / (p_{j+2} - p_{j-2}) - omega1), 0, 1),
// the ratio +inf where p_{j+2} = p_{j-2}.
// (The neighbour's weight, which needs pressures three cells away, beyond
// the ghost layers of the reconstructed cells, is not taken.)
__device__ inline double flatten_weight(const double *p, const double *un) {
    const double dp1 = p[3] - p[1];
    if (!(un[1] - un[3] > 0.0)) return 0.0;
    if (!(fabs(dp1) / fmin(p[3], p[1]) > CW_EPS_SHOCK)) return 0.0;
    const double dp2 = p[4] - p[0];
    // equal outer pressures: +inf in either direction of the line
    const double ratio = dp2 != 0.0 ? dp1 / dp2 : INFINITY;
    return fmax(0.0, fmin(1.0, CW_OMEGA2 * (ratio - CW_OMEGA1)));
}

// PPM with the steepening weight eta and the flattening weight flat.
__device__ inline void ppm_cw(const double *u, double eta, double flat, double &qp,
                              double &qm) {
    const double sixth = 1.0 / 6.0;
    const double s_m = mc_slope(u[0], u[1], u[2]);
    const double s_0 = mc_slope(u[1], u[2], u[3]);
    const double s_p = mc_slope(u[2], u[3], u[4]);
    const double u0 = u[2];
    qp = 0.5 * (u0 + u[3]) - (s_p - s_0) * sixth;
    qm = 0.5 * (u[1] + u0) - (s_0 - s_m) * sixth;
    if (eta > 0.0) {
        const double dm = u[1] + 0.5 * s_m;
        const double dp = u[3] - 0.5 * s_p;
        qm = qm * (1.0 - eta) + dm * eta;
        qp = qp * (1.0 - eta) + dp * eta;
    }
    if (flat > 0.0) {
        qm = flat * u0 + (1.0 - flat) * qm;
        qp = flat * u0 + (1.0 - flat) * qp;
    }
    if ((qp - u0) * (u0 - qm) <= 0.0) {
        qp = u0;
        qm = u0;
    } else {
        const double dq = qp - qm;
        const double m6 = 6.0 * (u0 - 0.5 * (qm + qp));
        if (dq * m6 > dq * dq) {
            qm = 3.0 * u0 - 2.0 * qp;
        } else if (-(dq * dq) > dq * m6) {
            qp = 3.0 * u0 - 2.0 * qm;
        }
    }
}

// One block per (subgrid, field, line); threads stride over the QCELL cells.
__global__ __launch_bounds__(256) void k_reconstruct(StepArgs a, const double *__restrict__ U,
                                                     double *__restrict__ Q,
                                                     const int64_t *__restrict__ q_offset) {
    const int per = NF_MAX * 13;
    const int s = blockIdx.x / per;
    const int r = blockIdx.x - s * per;
    const int f = r / 13;
    const int line = r - f * 13;
    if (s >= a.n_sub) return;
    int nf;
    int64_t off;
    if (!meta_ok(a, s, nf, off) || f >= nf) return;
    int dx, dy, dz;
    line_dir(line, dx, dy, dz);
    const int sp = 13 + line;          // slot of +d
    const int sm = 12 - line;          // slot of -d
    const int step = (dz * NB + dy) * NB + dx;
    const double *Uf = U + off + (int64_t)f * a.fstride;
    const double *Ur = U + off;                      // density
    double *Qf = Q + q_offset[s] + (int64_t)f * 26 * QCELL;
    const bool vel = a.vel && f >= 1 && f <= 3;
    const bool cw = a.steepen || a.flatten;
    for (int c = threadIdx.x; c < QCELL; c += blockDim.x) {
        int i = c % QN + 2, j = (c / QN) % QN + 2, k = c / (QN * QN) + 2;
        int ci = (k * NB + j) * NB + i;
        double qp, qm;
        if (cw) {
            double u[5], rho[5], p[5], un[5];
            for (int m = 0; m < 5; m++) {
                const int cm = ci + (m - 2) * step;
                rho[m] = Ur[cm];
                u[m] = vel ? Uf[cm] / rho[m] : Uf[cm];
                cell_p_un(a, Ur, cm, dx, dy, dz, p[m], un[m]);
            }
            const double eta = (a.steepen && f == 0) ? steepen_weight(a.gamma, rho, p) : 0.0;
            const double flat = a.flatten ? flatten_weight(p, un) : 0.0;
            ppm_cw(u, eta, flat, qp, qm);
            if (vel) {
                // the density's own values at the two points, with the same weights
                double rp, rm;
                ppm_cw(rho, a.steepen ? steepen_weight(a.gamma, rho, p) : 0.0, flat, rp, rm);
                qp = rp * qp;
                qm = rm * qm;
            }
        } else if (vel) {
            // velocity option: PPM of s / rho, times the point density (the
            // density's PPM is formed again here, as in its own block)
            double r[5], w[5];
            for (int m = 0; m < 5; m++) {
                const int cm = ci + (m - 2) * step;
                r[m] = Ur[cm];
                w[m] = Uf[cm] / r[m];
            }
            double rp, rm;
            ppm(r[0], r[1], r[2], r[3], r[4], rp, rm);
            ppm(w[0], w[1], w[2], w[3], w[4], qp, qm);
            qp = rp * qp;
            qm = rm * qm;
        } else {
            ppm(Uf[ci - 2 * step], Uf[ci - step], Uf[ci], Uf[ci + step], Uf[ci + 2 * step], qp,
                qm);
        }
        Qf[sp * QCELL + c] = qp;
        Qf[sm * QCELL + c] = qm;
    }
}

// ---- point state -------------------------------------------------------------

struct PointState {
    double un, p, cs;
    int bits;
};

__device__ inline PointState point_state(const StepArgs &a, double rho, double sx, double sy,
                                         double sz, double E, double tau, int axis) {
    PointState st;
    double r = 1.0 / rho;
    double vx = sx * r, vy = sy * r, vz = sz * r;
    double ek = 0.5 * ((sx * vx + sy * vy) + sz * vz);
    double ei = E - ek;
    if (ei < a.de_switch * E) ei = pow(tau, a.gamma);
    double p = (a.gamma - 1.0) * ei;
    st.cs = sqrt((a.gamma * p) * r);
    st.un = axis == 0 ? vx : (axis == 1 ? vy : vz);
    st.p = p;
    st.bits = (rho <= 0.0 ? 1 : 0) | (p <= 0.0 ? 2 : 0);
    return st;
}

// Physical flux of field f along axis at a point with state (un, p); V_f is the
// field's own value, s_axis the normal momentum (used by the density flux).
__device__ inline double phys_flux(int f, int axis, double vf, double s_axis, double un,
                                   double p) {
    if (f == 0) return s_axis;
    if (f <= 3) {
        double v = vf * un;
        if (f - 1 == axis) v = v + p;
        return v;
    }
    if (f == 4) return (vf + p) * un;
    return vf * un;
}

__device__ inline void block_reduce_max_or(double &m, int &bits) {
    __shared__ double sm[16];
    __shared__ int sb[16];
    for (int o = 32; o > 0; o >>= 1) {
        m = fmax(m, __shfl_xor(m, o));
        bits |= __shfl_xor(bits, o);
    }
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sm[w] = m;
        sb[w] = bits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < (int)(blockDim.x >> 6); q++) {
            m = fmax(m, sm[q]);
            bits |= sb[q];
        }
    }
}

__global__ void k_init_outputs(int n, double *amax, int32_t *status) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) {
        amax[s] = 0.0;
        if (status) status[s] = 0;
    }
}

// One block per (subgrid, 256-face chunk); FLUX_CHUNKS chunks cover the
// 3 x NFACE faces.
constexpr int FLUX_CHUNKS = (3 * NFACE + 255) / 256;

__global__ __launch_bounds__(256) void k_flux(StepArgs a, const double *__restrict__ Q,
                                              const int64_t *__restrict__ q_offset,
                                              double *__restrict__ F,
                                              const int64_t *__restrict__ f_offset,
                                              double *amax, int32_t *status) {
    const int s = blockIdx.x / FLUX_CHUNKS;
    const int chunk = blockIdx.x - s * FLUX_CHUNKS;
    if (s >= a.n_sub) return;
    int nf;
    int64_t off;
    if (!meta_ok(a, s, nf, off)) {
        if (chunk == 0 && threadIdx.x == 0 && status) atomicOr(&status[s], (int)HYDRO_STATUS_BADMETA);
        return;
    }
    const double *Qs = Q + q_offset[s];
    double *Fs = F + f_offset[s];
    const int face = chunk * 256 + threadIdx.x;
    double af = 0.0;
    int bits = 0;
    if (face < 3 * NFACE) {
        const int axis = face / NFACE;
        const int idx = face - axis * NFACE;
        constexpr int n = NSUB, n1 = NSUB + 1;
        int cl[3];
        if (axis == 0) {
            cl[0] = 2 + idx % n1; cl[1] = NG + (idx / n1) % n; cl[2] = NG + idx / (n * n1);
        } else if (axis == 1) {
            cl[0] = NG + idx % n; cl[1] = 2 + (idx / n) % n1; cl[2] = NG + idx / (n * n1);
        } else {
            cl[0] = NG + idx % n; cl[1] = NG + (idx / n) % n; cl[2] = 2 + idx / (n * n);
        }
        int cr[3] = {cl[0], cl[1], cl[2]};
        cr[axis] += 1;
        const int b = axis == 0 ? 1 : 0;
        const int b2 = axis == 2 ? 1 : 2;
        const int qcl = qcell(cl[0], cl[1], cl[2]);
        const int qcr = qcell(cr[0], cr[1], cr[2]);
        int sl[9], sr[9];
        for (int t = 0; t < 9; t++) {
            int d[3] = {0, 0, 0};
            d[b] = t % 3 - 1;
            d[b2] = t / 3 - 1;
            d[axis] = 1;
            sl[t] = dir_slot(d[0], d[1], d[2]);
            d[axis] = -1;
            sr[t] = dir_slot(d[0], d[1], d[2]);
        }
        // pass 1: point states on both sides and the face's one-sided speeds
        double unL[9], pL[9], unR[9], pR[9];
        double lam_p = -INFINITY, lam_m = INFINITY;
        for (int t = 0; t < 9; t++) {
            const double *qL = Qs + (int64_t)sl[t] * QCELL + qcl;
            const double *qR = Qs + (int64_t)sr[t] * QCELL + qcr;
            const int64_t fs = 26 * QCELL;
            PointState L = point_state(a, qL[0], qL[fs], qL[2 * fs], qL[3 * fs], qL[4 * fs],
                                       qL[5 * fs], axis);
            PointState R = point_state(a, qR[0], qR[fs], qR[2 * fs], qR[3 * fs], qR[4 * fs],
                                       qR[5 * fs], axis);
            bits |= L.bits | R.bits;
            unL[t] = L.un; pL[t] = L.p;
            unR[t] = R.un; pR[t] = R.p;
            lam_p = fmax(lam_p, fmax(L.un + L.cs, R.un + R.cs));
            lam_m = fmin(lam_m, fmin(L.un - L.cs, R.un - R.cs));
        }
        double ap = fmax(0.0, lam_p);
        double am = fmin(0.0, lam_m);
        if (a.sym) {   // one speed for both directions
            const double sa = fmax(ap, -am);
            ap = sa;
            am = -sa;
        }
        const double inv = 1.0 / (ap - am);
        const double apam = ap * am;
        const double sixth = 1.0 / 6.0;
        const double two_thirds = 4.0 / 6.0;
        // pass 2: per field, point fluxes and the nested Simpson average
        for (int f = 0; f < nf; f++) {
            double H[9];
            for (int t = 0; t < 9; t++) {
                const double *qL = Qs + ((int64_t)f * 26 + sl[t]) * QCELL + qcl;
                const double *qR = Qs + ((int64_t)f * 26 + sr[t]) * QCELL + qcr;
                double vl = qL[0], vr = qR[0];
                double saL = 0.0, saR = 0.0;
                if (f == 0) {
                    saL = Qs[((int64_t)(1 + axis) * 26 + sl[t]) * QCELL + qcl];
                    saR = Qs[((int64_t)(1 + axis) * 26 + sr[t]) * QCELL + qcr];
                }
                double FL = phys_flux(f, axis, vl, saL, unL[t], pL[t]);
                double FR = phys_flux(f, axis, vr, saR, unR[t], pR[t]);
                H[t] = (((ap * FL) - (am * FR)) + (apam * (vr - vl))) * inv;
            }
            double r0 = sixth * (H[0] + H[2]) + two_thirds * H[1];
            double r1 = sixth * (H[3] + H[5]) + two_thirds * H[4];
            double r2 = sixth * (H[6] + H[8]) + two_thirds * H[7];
            double fb = sixth * (r0 + r2) + two_thirds * r1;
            Fs[((int64_t)f * 3 + axis) * NFACE + idx] = fb;
            if (!isfinite(fb)) bits |= HYDRO_STATUS_NONFINITE;
        }
        af = fmax(ap, -am);
        if (!isfinite(af)) bits |= HYDRO_STATUS_NONFINITE;
        af = af + 0.0;      // -0 -> +0 so the bit pattern orders like the value
    }
    block_reduce_max_or(af, bits);
    if (threadIdx.x == 0) {
        // non-negative doubles order like their bit patterns (NaN above +inf)
        atomicMax(reinterpret_cast<unsigned long long *>(&amax[s]),
                  (unsigned long long)__double_as_longlong(af));
        if (status && bits) atomicOr(&status[s], bits);
    }
}

// One block per (subgrid, field, 256 of the interior cells).
constexpr int DIV_CHUNKS = NINT / 256;

__global__ __launch_bounds__(256) void k_divergence(StepArgs a, const double *__restrict__ F,
                                                    const int64_t *__restrict__ f_offset,
                                                    const double *__restrict__ U_in,
                                                    double *__restrict__ U_out) {
    const int per = NF_MAX * DIV_CHUNKS;
    const int s = blockIdx.x / per;
    const int r = blockIdx.x - s * per;
    const int f = r / DIV_CHUNKS;
    if (s >= a.n_sub) return;
    int nf;
    int64_t off;
    if (!meta_ok(a, s, nf, off) || f >= nf) return;
    const int c = (r - f * DIV_CHUNKS) * 256 + threadIdx.x;
    const int i = NG + c % NSUB, j = NG + (c / NSUB) % NSUB, k = NG + c / (NSUB * NSUB);
    const double lam = a.dt / a.h[s];
    const double *Fs = F + f_offset[s] + (int64_t)f * 3 * NFACE;
    const double *Fx = Fs, *Fy = Fs + NFACE, *Fz = Fs + 2 * NFACE;
    double dfx = Fx[face_idx(0, i, j, k)] - Fx[face_idx(0, i - 1, j, k)];
    double dfy = Fy[face_idx(1, i, j, k)] - Fy[face_idx(1, i, j - 1, k)];
    double dfz = Fz[face_idx(2, i, j, k)] - Fz[face_idx(2, i, j, k - 1)];
    const int64_t ci = off + (int64_t)f * a.fstride + (k * NB + j) * NB + i;
    U_out[ci] = U_in[ci] - lam * ((dfx + dfy) + dfz);
}

}  // namespace

hipError_t launch_plain_reconstruct(const StepArgs &a, const double *U, double *Q,
                                    const int64_t *q_offset, hipStream_t st) {
    if (a.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reconstruct, dim3(a.n_sub * NF_MAX * 13), dim3(256), 0, st, a, U, Q,
                       q_offset);
    return hipGetLastError();
}

hipError_t launch_plain_flux(const StepArgs &a, const double *Q, const int64_t *q_offset,
                             double *F, const int64_t *f_offset, double *amax,
                             int32_t *status, hipStream_t st) {
    if (a.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_outputs, dim3((a.n_sub + 255) / 256), dim3(256), 0, st, a.n_sub,
                       amax, status);
    hipLaunchKernelGGL(k_flux, dim3(a.n_sub * FLUX_CHUNKS), dim3(256), 0, st, a, Q, q_offset, F,
                       f_offset, amax, status);
    return hipGetLastError();
}

hipError_t launch_plain_divergence(const StepArgs &a, const double *F, const int64_t *f_offset,
                                   const double *U_in, double *U_out, hipStream_t st) {
    if (a.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_divergence, dim3(a.n_sub * NF_MAX * DIV_CHUNKS), dim3(256), 0, st, a, F,
                       f_offset, U_in, U_out);
    return hipGetLastError();
}

}  // namespace hydro
