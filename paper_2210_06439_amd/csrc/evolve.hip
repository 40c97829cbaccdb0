// evolve.hip -- device-resident time integration around the fused stage:
// ghost fill from neighbour interiors, the batch-wide CFL step size, and the
// SSP-RK3 stage combination.  Sec. V (Test 2): one time step holds three
// hydro iterations; Test 1 names time-step size determination and ghost
// exchange as part of every step; Test 3 finds ghost handling to be where
// much of the hydro time goes on a CPU.
#include "hydro_internal.hpp"

namespace hydro {
namespace {

constexpr int NI = NSUB;   // interior cells per dimension

// Source index along one axis of a ghost cell at index i (direction d):
// inside the interior (d == 0) the index itself; toward a neighbour its
// interior cell N cells back; at a clamped boundary the nearest interior cell.
__device__ __forceinline__ int ghost_src(int i, int d, bool clamp) {
    if (d == 0) return i;
    if (clamp) return i < NG ? NG : NG + NI - 1;
    return i - NI * d;
}

__device__ __forceinline__ int dir_of(int i) { return i < NG ? -1 : (i >= NG + NI ? 1 : 0); }

// The ghost cells of a block (2232 for 14^3, 6552 for 22^3), each packed as
// cell index (14 bits) and neighbour direction slot (5 bits), built once per
// block in LDS.
constexpr int NGHOST = NCELL - NI * NI * NI;
constexpr int CELL_BITS = 14;
static_assert(NCELL <= (1 << CELL_BITS), "cell index must fit its field");

// One block per (subgrid, field group): every ghost cell is copied from the
// interior cell that the map names.  Only interior cells are read and only
// ghost cells written, so the fill is safe in place.  Threads walk the ghost
// list, so consecutive threads copy consecutive cells of a row.
__global__ __launch_bounds__(512) void k_fill_ghosts(int n_sub, int fstride,
                                                     const int64_t *__restrict__ offset,
                                                     const int32_t *__restrict__ n_species,
                                                     const int32_t *__restrict__ src,
                                                     const int32_t *__restrict__ mode,
                                                     double *U, int32_t *status) {
    __shared__ int ghost[NGHOST];
    __shared__ int64_t src_off[27];
    __shared__ int src_mode[27];
    __shared__ int src_nf[27];
    const int s = blockIdx.x;
    const int ns = n_species[s];
    const int64_t off = offset[s];
    if (ns < 0 || ns > 5 || off < 0) return;
    const int nf = 6 + ns;
    // ghost list: cell c is a ghost iff some index is outside [NG, NG + NI)
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int i = c % NB, j = (c / NB) % NB, k = c / NPLANE;
        const int dx = dir_of(i), dy = dir_of(j), dz = dir_of(k);
        if ((dx | dy | dz) == 0) continue;
        // rank of c among ghosts: cells before c minus interior cells before c
        const int kk = k < NG ? 0 : (k >= NG + NI ? NI : k - NG);
        const int jj = j < NG ? 0 : (j >= NG + NI ? NI : j - NG);
        const int ii = i < NG ? 0 : (i >= NG + NI ? NI : i - NG);
        int inner = kk * NI * NI;                       // interior cells in planes below
        if (k >= NG && k < NG + NI) inner += jj * NI + ((j >= NG && j < NG + NI) ? ii : 0);
        const int n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
        ghost[c - inner] = c | (n << CELL_BITS);
    }
    if (threadIdx.x < 27) {
        const int sb = src[s * 27 + threadIdx.x];
        const bool ok = threadIdx.x != 13 && sb >= 0 && sb < n_sub;
        const int ns2 = ok ? n_species[sb] : -1;
        const int64_t off2 = ok ? offset[sb] : -1;
        const bool good = ok && ns2 >= 0 && ns2 <= 5 && off2 >= 0;
        src_off[threadIdx.x] = good ? off2 : -1;
        src_nf[threadIdx.x] = good ? 6 + ns2 : 0;
        src_mode[threadIdx.x] = mode[s * 27 + threadIdx.x];
    }
    __syncthreads();
    int bad = 0;
    for (int e = threadIdx.x; e < nf * NGHOST; e += blockDim.x) {
        const int f = e / NGHOST;
        const int g = ghost[e - f * NGHOST];
        const int c = g & ((1 << CELL_BITS) - 1), n = g >> CELL_BITS;
        const int64_t o2 = src_off[n];
        if (o2 < 0 || f >= src_nf[n]) {
            bad = 1;
            continue;
        }
        const int m = src_mode[n];
        const int i = c % NB, j = (c / NB) % NB, k = c / NPLANE;
        const int dx = n % 3 - 1, dy = (n / 3) % 3 - 1, dz = n / 9 - 1;
        const int si = ghost_src(i, dx, m & 1), sj = ghost_src(j, dy, m & 2),
                  sk = ghost_src(k, dz, m & 4);
        U[off + (int64_t)f * fstride + c] = U[o2 + (int64_t)f * fstride + (sk * NB + sj) * NB + si];
    }
    if (bad && status) atomicOr(&status[s], (int)HYDRO_STATUS_BADMETA);
}

// dt = cfl * min_s h_s / amax_s, cut so that the clock lands exactly on
// t_end; clock = {t, dt, steps taken with dt > 0}.  One block.
__global__ __launch_bounds__(1024) void k_cfl_dt(int n_sub, const double *__restrict__ h,
                                                 const double *__restrict__ amax, double cfl,
                                                 double t_end, double *clock) {
    __shared__ double red[16];
    double m = INFINITY;
    for (int s = threadIdx.x; s < n_sub; s += blockDim.x) {
        const double a = amax[s];
        if (a > 0.0) m = fmin(m, h[s] / a);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = fmin(m, red[w]);
        double t = clock[0];
        const double rem = t_end - t;
        double dt = cfl * m;
        if (!(rem > 0.0)) {
            dt = 0.0;
        } else if (!(dt < rem)) {
            dt = rem;
            t = t_end;
        } else {
            t = t + dt;
        }
        if (!isfinite(dt)) dt = 0.0;
        clock[0] = t;
        clock[1] = dt;
        if (dt > 0.0) clock[2] += 1.0;
    }
}

// U_out = a U0 + b (Uk + dt R) on the interior, dt = clock[1]; with dt == 0
// the stage is the identity (U_out = U0), which makes a whole step a no-op.
__global__ __launch_bounds__(512) void k_rk_update(int fstride, const int64_t *__restrict__ offset,
                                                   const int32_t *__restrict__ n_species,
                                                   double a, const double *U0, double b,
                                                   const double *Uk, const double *R,
                                                   const double *__restrict__ clock,
                                                   double *Uo) {
    const int s = blockIdx.x, f = blockIdx.y;
    const int ns = n_species[s];
    const int64_t off = offset[s];
    if (ns < 0 || ns > 5 || off < 0 || f >= 6 + ns) return;
    const double dt = clock[1];
    for (int t = threadIdx.x; t < NINT; t += blockDim.x) {
        const int i = NG + t % NI, j = NG + (t / NI) % NI, k = NG + t / (NI * NI);
        const int64_t idx = off + (int64_t)f * fstride + (k * NB + j) * NB + i;
        const double u0 = U0[idx];
        Uo[idx] = dt == 0.0 ? u0 : a * u0 + b * (Uk[idx] + dt * R[idx]);
    }
}

// Entropy-tracer re-synchronisation: tau = e_i^(1/gamma) where the internal
// energy from E is reliable (e_i not below de_switch * E).  One block per
// subgrid, threads striding over the interior cells; evaluated in the written order (no
// contraction), so the switch decides exactly as in the point state.
__global__ __launch_bounds__(512) void k_tau_resync(StepArgs a, double *U) {
#pragma clang fp contract(off)
    const int s = blockIdx.x;
    const int ns = a.n_species[s];
    const int64_t off = a.offset[s];
    if (ns < 0 || ns > 5 || off < 0) return;
    const int64_t fs = a.fstride;
    for (int t = threadIdx.x; t < NINT; t += blockDim.x) {
        const int i = NG + t % NI, j = NG + (t / NI) % NI, k = NG + t / (NI * NI);
        double *u = U + off + (k * NB + j) * NB + i;
        const double rho = u[0], sx = u[fs], sy = u[2 * fs], sz = u[3 * fs], E = u[4 * fs];
        const double r = 1.0 / rho;
        const double vx = sx * r, vy = sy * r, vz = sz * r;
        const double ek = 0.5 * ((sx * vx + sy * vy) + sz * vz);
        const double ei = E - ek;
        if (!(ei < a.de_switch * E)) u[5 * fs] = pow(ei, 1.0 / a.gamma);
    }
}

}  // namespace

hipError_t launch_tau_resync(const StepArgs &a, double *U, hipStream_t st) {
    if (a.n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tau_resync, dim3(a.n_sub), dim3(512), 0, st, a, U);
    return hipGetLastError();
}

hipError_t launch_fill_ghosts(int n_sub, int fstride, const int64_t *offset,
                              const int32_t *n_species, const int32_t *src, const int32_t *mode,
                              double *U, int32_t *status, hipStream_t st) {
    if (n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_ghosts, dim3(n_sub), dim3(512), 0, st, n_sub, fstride, offset,
                       n_species, src, mode, U, status);
    return hipGetLastError();
}

hipError_t launch_cfl_dt(int n_sub, const double *h, const double *amax, double cfl,
                         double t_end, double *clock, hipStream_t st) {
    hipLaunchKernelGGL(k_cfl_dt, dim3(1), dim3(1024), 0, st, n_sub, h, amax, cfl, t_end, clock);
    return hipGetLastError();
}

hipError_t launch_rk_update(int n_sub, int fstride, const int64_t *offset,
                            const int32_t *n_species, double a, const double *U0, double b,
                            const double *Uk, const double *R, const double *clock, double *Uo,
                            hipStream_t st) {
    if (n_sub == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rk_update, dim3(n_sub, NF_MAX), dim3(512), 0, st, fstride, offset,
                       n_species, a, U0, b, Uk, R, clock, Uo);
    return hipGetLastError();
}

}  // namespace hydro
