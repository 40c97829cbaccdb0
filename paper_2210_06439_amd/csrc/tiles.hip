// tiles.hip -- the fused step for 16^3 subgrids.
//
// The step is local: every interior cell depends only on the cells within
// three of it (Sec. II, "Data-Structure", reconstruction and flux stencils),
// so a 16^3 subgrid and the eight 8^3 subgrids that tile it, cut with their
// ghosts from the same (16+6)^3 block, have the same interiors, the same
// largest face speed and the same status bits.  The fused kernel is written
// for 8^3 subgrids (one 64-lane wave per 8 x 8 plane); this library compiles
// it with the 16^3 block's row pitch, so it reads each tile's 14^3 window
// straight from the block and writes the tile's interior into the output
// block.  This file lists the tiles and reduces their speeds and status
// words per subgrid.
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "hydro_internal.hpp"

namespace hydro {

static_assert(NSUB == 16, "the tiled fused step serves the 16^3 build");

namespace {

constexpr int TN = 8;                    // tile interior

__device__ __forceinline__ bool meta_bad(int nsp, int64_t o) {
    return nsp < 0 || nsp > 5 || o < 0 || (o & 1);
}

// Tile t of subgrid s = t / 8 lies at (8 tx, 8 ty, 8 tz) of its block, with
// t % 8 = 4 tz + 2 ty + tx; its metadata: the offset of its 14^3 window in
// the block, the subgrid's h and species count (-1 when the subgrid's
// metadata is invalid, which the fused kernel reports as such).
__global__ void k_tile_meta(int n, const int64_t *__restrict__ off, const double *__restrict__ h,
                            const int32_t *__restrict__ ns, int64_t *toff, double *th,
                            int32_t *tns) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 8 * n) return;
    const int s = t >> 3;
    const int nsp = ns[s];
    const int64_t o = off[s];
    const int tx = t & 1, ty = (t >> 1) & 1, tz = (t >> 2) & 1;
    const bool bad = meta_bad(nsp, o);
    toff[t] = bad ? 0 : o + ((TN * tz) * NB + TN * ty) * NB + TN * tx;
    th[t] = h[s];
    tns[t] = bad ? -1 : nsp;
}

// The subgrid's largest face speed and status word from its eight tiles'
// (the maximum as the fused kernel forms it, fmax; the status bits ORed).
__global__ void k_tile_reduce(int n, const double *__restrict__ tam,
                              const int32_t *__restrict__ tst, double *amax, int32_t *status) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    double m = tam[8 * s];
    int b = tst[8 * s];
    for (int q = 1; q < 8; q++) {
        m = fmax(m, tam[8 * s + q]);
        b |= tst[8 * s + q];
    }
    amax[s] = m;
    if (status) status[s] = b;
}

// Tile metadata and per-tile results per (device, stream), grown on demand.
struct TileWork {
    int cap = 0;                 // subgrids
    double *th = nullptr, *tam = nullptr;
    int64_t *toff = nullptr;
    int32_t *tns = nullptr, *tst = nullptr;
};
std::mutex g_tw_mu;
std::map<std::pair<int, void *>, TileWork> g_tw;

void tile_free(TileWork &w) {
    hipFree(w.th);
    hipFree(w.tam);
    hipFree(w.toff);
    hipFree(w.tns);
    hipFree(w.tst);
    w = TileWork();
}

hipError_t tile_work(void *stream, int n, TileWork **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tw_mu);
    TileWork &w = g_tw[std::make_pair(dev, stream)];
    if (w.cap < n) {
        if (w.cap) {
            // the old buffers may still be in use by launches on the stream
            if ((e = hipStreamSynchronize(static_cast<hipStream_t>(stream))) != hipSuccess) return e;
            tile_free(w);
        }
        const size_t nt = (size_t)8 * n;
        if ((e = hipMalloc(&w.th, nt * sizeof(double))) == hipSuccess &&
            (e = hipMalloc(&w.tam, nt * sizeof(double))) == hipSuccess &&
            (e = hipMalloc(&w.toff, nt * sizeof(int64_t))) == hipSuccess &&
            (e = hipMalloc(&w.tns, nt * sizeof(int32_t))) == hipSuccess &&
            (e = hipMalloc(&w.tst, nt * sizeof(int32_t))) == hipSuccess) {
            w.cap = n;
        } else {
            tile_free(w);
            return e;
        }
    }
    *out = &w;
    return hipSuccess;
}

// The launch shape of the tile batch: one sweep per tile (the split and
// dynamic shapes need scratch), persistent with one workgroup per CU and the
// tiles in reverse order, the fastest such shape on thousands of 8^3 blocks.
int tile_variant() {
    static const int v = [] {
        for (int i = 0; i < fused_variant_count(); i++)
            if (!std::strcmp(fused_variant_name(i), "persistent-1x-rev")) return i;
        return 1;
    }();
    return v;
}

}  // namespace

int64_t tiled_work_bytes(int dev) {
    std::lock_guard<std::mutex> lk(g_tw_mu);
    int64_t b = 0;
    for (auto &kv : g_tw)
        if (kv.first.first == dev)
            b += (int64_t)kv.second.cap * 8 *
                 (2 * sizeof(double) + sizeof(int64_t) + 2 * sizeof(int32_t));
    return b;
}

hipError_t launch_tiled_step(const StepArgs &a, const double *U_in, double *U_out, double *amax,
                             int32_t *status, void *stream) {
    const int n = a.n_sub;
    if (n == 0) return hipSuccess;
    if (fused_global_pitch() != NB) return hipErrorInvalidValue;   // built for other blocks
    TileWork *w = nullptr;
    hipError_t e = tile_work(stream, n, &w);
    if (e != hipSuccess) return e;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nt = 8 * n;
    hipLaunchKernelGGL(k_tile_meta, dim3((nt + 255) / 256), dim3(256), 0, st, n, a.offset, a.h,
                       a.n_species, w->toff, w->th, w->tns);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the tiles as a batch of 8^3 subgrids in the blocks' layout (the output
    // at the same offsets of U_out), in a one-sweep shape (no scratch)
    StepArgs ta = a;
    ta.n_sub = nt;
    ta.offset = w->toff;
    ta.out_offset = nullptr;
    ta.h = w->th;
    ta.n_species = w->tns;
    ta.scratch = nullptr;
    if ((e = launch_fused_step(ta, U_in, U_out, w->tam, w->tst, tile_variant(), st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_tile_reduce, dim3((n + 255) / 256), dim3(256), 0, st, n, w->tam, w->tst,
                       amax, status);
    return hipGetLastError();
}

}  // namespace hydro
