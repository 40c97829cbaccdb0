// api.hip -- the C ABI of the hydro library: argument checks, launches,
// the autotuner's cache and captured hipGraph plans.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "hydro_internal.hpp"

using namespace hydro;

namespace {

thread_local char g_err[256];
thread_local hipError_t g_last_hip = hipSuccess;

int fail_hip(hipError_t e) {
    g_last_hip = e;
    return HYDRO_ELAUNCH;
}

// The device must be a gfx950; checked once per device.
int check_device() {
    static std::mutex mu;
    static std::unordered_map<int, int> ok;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    std::lock_guard<std::mutex> lk(mu);
    auto it = ok.find(dev);
    if (it != ok.end()) return it->second;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail_hip(e);
    int r = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0 ? HYDRO_OK : HYDRO_ENODEV;
    ok[dev] = r;
    return r;
}

int check_batch(const hydro_batch *b) {
    if (!b) return HYDRO_EINVAL;
    if (b->n_sub < 0 || b->fstride < NCELL || (b->fstride & 1)) return HYDRO_EINVAL;
    if (b->n_sub > 0 && (!b->offset || !b->h || !b->n_species)) return HYDRO_EINVAL;
    return HYDRO_OK;
}

int check_common(const hydro_params *p, const hydro_batch *b) {
    if (!p || check_batch(b)) return HYDRO_EINVAL;
    if (p->flags & ~(uint32_t)(HYDRO_FLAG_KT_SYMMETRIC | HYDRO_FLAG_VELOCITY | HYDRO_FLAG_STEEPEN |
                               HYDRO_FLAG_FLATTEN))
        return HYDRO_EINVAL;
    return HYDRO_OK;
}

// The fused kernel covers 8^3 subgrids only: its entry points refuse other
// builds.
int check_fused(const hydro_params *p, const hydro_batch *b) {
    int rc = check_common(p, b);
    if (rc) return rc;
    if (NSUB != 8) return HYDRO_EINVAL;
    return HYDRO_OK;
}

bool aligned8(const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 7u) == 0; }

// ---- autotuner cache: power-of-two bucket of n_sub -> variant --------------

std::mutex g_tune_mu;
std::unordered_map<int, int> g_tuned;
bool g_tune_loaded = false;

int bucket_of(int n_sub) {
    int b = 0;
    while ((1 << b) < n_sub && b < 30) b++;
    return b;
}

const char *tune_file() { return std::getenv("HYDRO_TUNE_CACHE"); }

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *fn = tune_file();
    if (!fn) return;
    FILE *f = std::fopen(fn, "r");
    if (!f) return;
    char arch[32];
    int bucket, variant;
    while (std::fscanf(f, "%31s %d %d", arch, &bucket, &variant) == 3)
        if (std::strcmp(arch, "gfx950") == 0 && variant >= 0 && variant < fused_variant_count())
            g_tuned[bucket] = variant;
    std::fclose(f);
}

void tune_save_locked() {
    const char *fn = tune_file();
    if (!fn) return;
    std::string tmp = std::string(fn) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    for (auto &kv : g_tuned) std::fprintf(f, "gfx950 %d %d\n", kv.first, kv.second);
    std::fclose(f);
    std::rename(tmp.c_str(), fn);
}

// ---- scratch of the split and dynamic launch shapes -----------------------
//
// The library keeps one scratch buffer per (device, stream) for the eager
// calls, zero-filled when allocated (the kernel leaves it zero after every
// launch).  Plans and RK3 graphs own their own.  The first call that needs
// scratch on a stream allocates it, so that call must not be made while the
// stream is being captured.  That first buffer covers kScratchMinSub
// subgrids (about 1 MiB), so a stream whose batch sizes vary (a serving
// loop's ticks) does not grow it: growing synchronizes the stream and frees
// the old buffer, a stall of the whole loop.  Beyond that it grows to at
// least twice its size.

struct Scratch {
    uint32_t *ptr = nullptr;
    int64_t bytes = 0;
};

std::mutex g_ws_mu;
std::map<std::pair<int, void *>, Scratch> g_ws;
constexpr int kScratchMinSub = 65536;

int alloc_scratch(int64_t bytes, uint32_t **out) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)bytes);
    if (e == hipSuccess) e = hipMemset(p, 0, (size_t)bytes);
    if (e != hipSuccess) {
        if (p) hipFree(p);
        return fail_hip(e);
    }
    *out = static_cast<uint32_t *>(p);
    return HYDRO_OK;
}

// Scratch for `n_sub` subgrids on the current device and `stream`.
int stream_scratch(void *stream, int n_sub, uint32_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    const int64_t need = fused_scratch_bytes(n_sub);
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Scratch &w = g_ws[std::make_pair(dev, stream)];
    if (w.bytes < need) {
        if (w.ptr) {
            // the old buffer may still be in use by launches on the stream
            e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
            if (e != hipSuccess) return fail_hip(e);
            hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        const int64_t old = w.bytes;
        int64_t bytes = fused_scratch_bytes(kScratchMinSub);
        if (bytes < 2 * old) bytes = 2 * old;
        if (bytes < need) bytes = need;
        int rc = alloc_scratch(bytes, &w.ptr);
        if (rc) return rc;
        w.bytes = bytes;
    }
    *out = w.ptr;
    return HYDRO_OK;
}

// ---- scratch of hydro_step_noalloc ------------------------------------------
//
// A file-scope device array, one copy per GPU, held until the process ends:
// the split and dynamic launch shapes' scratch for up to
// HYDRO_NOALLOC_MAX_SUB subgrids.  Host code never passes `scratch` itself
// to a kernel (on the host it only names the symbol): its device address is
// looked up once per device and kept in g_noalloc.

constexpr int64_t kNoallocBytes = fused_scratch_bytes_for(HYDRO_NOALLOC_MAX_SUB);
static __device__ __align__(256) uint32_t scratch[kNoallocBytes / 4];

std::mutex g_noalloc_mu;
std::unordered_map<int, uint32_t *> g_noalloc;

// Device address of this device's `scratch` (looked up on its first use).
int noalloc_scratch(uint32_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e);
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc.find(dev);
    if (it == g_noalloc.end()) {
        uint32_t *ptr = nullptr;
        e = hipGetSymbolAddress(reinterpret_cast<void **>(&ptr), HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol);
        it = g_noalloc.emplace(dev, ptr).first;
    }
    *out = it->second;
    return HYDRO_OK;
}

// Zero n words (a kernel, not a memset node, so that a caller may capture it).
__global__ void k_clear_words(uint32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// ---- block copies (hydro_copy_blocks) ---------------------------------------
//
// Workgroup g copies chunk g % chunks of pair g / chunks: one read of the
// source row's chunk, written to one or two destination rows.  vec2: rows and
// buffers 16-byte aligned, so the chunk moves as double2.
constexpr int kCopyThreads = 256;
constexpr int64_t kCopyChunk = 2048;      // doubles per workgroup

__global__ __launch_bounds__(kCopyThreads) void k_copy_blocks(
    const double *__restrict__ src, int64_t src_rows, const int64_t *__restrict__ src_row,
    double *__restrict__ dst, int64_t dst_rows, const int64_t *__restrict__ d0,
    const int64_t *__restrict__ d1, int64_t row_elems, int chunks, int vec2) {
    const int64_t i = blockIdx.x / chunks;
    const int64_t c = blockIdx.x % chunks;
    const int64_t r = src_row[i], a = d0[i], b = d1 ? d1[i] : -1;
    if (r < 0 || r >= src_rows) return;
    const bool wa = a >= 0 && a < dst_rows, wb = b >= 0 && b < dst_rows;
    if (!wa && !wb) return;
    const int64_t lo = c * kCopyChunk;
    const int64_t hi = lo + kCopyChunk < row_elems ? lo + kCopyChunk : row_elems;
    const double *s = src + r * row_elems;
    double *da = dst + (wa ? a : 0) * row_elems, *db = dst + (wb ? b : 0) * row_elems;
    if (vec2) {
        const double2 *s2 = reinterpret_cast<const double2 *>(s);
        double2 *da2 = reinterpret_cast<double2 *>(da), *db2 = reinterpret_cast<double2 *>(db);
        for (int64_t e = lo / 2 + threadIdx.x; e < hi / 2; e += kCopyThreads) {
            const double2 v = s2[e];
            if (wa) da2[e] = v;
            if (wb) db2[e] = v;
        }
    } else {
        for (int64_t e = lo + threadIdx.x; e < hi; e += kCopyThreads) {
            const double v = s[e];
            if (wa) da[e] = v;
            if (wb) db[e] = v;
        }
    }
}

// Launch the fused step in `variant`, attaching the stream's scratch when
// the step needs it.
int launch_step(StepArgs a, const double *U_in, double *U_out, double *amax, int32_t *status,
                int variant, void *stream) {
    if (fused_needs_scratch(a, variant) && !a.scratch) {
        int rc = stream_scratch(stream, a.n_sub, &a.scratch);
        if (rc) return rc;
    }
    hipError_t e = launch_fused_step(a, U_in, U_out, amax, status, variant,
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

}  // namespace

struct hydro_plan {
    StepArgs args;
    const double *U_in;
    double *U_out;
    double *amax;
    int32_t *status;
    int variant;
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint32_t *scratch;   // owned
};

struct hydro_rk3 {
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint32_t *scratch;   // owned
};

namespace {

// Whether the batch holds no subgrid without species, read once when a plan
// or an RK3 graph is made: its steps then launch the 11-field kernel alone,
// which sweeps every subgrid itself when it runs alone (so a later change of
// the species counts stays correct).
int batch_unpaired(const hydro_batch *b, int32_t *out) {
    std::vector<int32_t> ns((size_t)b->n_sub);
    hipError_t e = hipMemcpy(ns.data(), b->n_species, ns.size() * sizeof(int32_t),
                             hipMemcpyDefault);
    if (e != hipSuccess) return fail_hip(e);
    *out = 1;
    for (int32_t v : ns)
        if (v == 0) *out = 0;
    return HYDRO_OK;
}

// Record the plan's step (the fused kernels of its launch shape) into a graph
// and make it the plan's: a new executable graph, or an update of the one the
// plan has (whose launches may still be in flight).
hipError_t plan_build(hydro_plan *p) {
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = launch_fused_step(p->args, p->U_in, p->U_out, p->amax, p->status,
                                          p->variant, cs);
        e = hipStreamEndCapture(cs, &g);
        if (e1 != hipSuccess) e = e1;
    }
    hipStreamDestroy(cs);
    if (e == hipSuccess && p->exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res;
        e = hipGraphExecUpdate(p->exec, g, &bad, &res);
    } else if (e == hipSuccess) {
        e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return e;
    }
    if (p->graph) hipGraphDestroy(p->graph);
    p->graph = g;
    return hipSuccess;
}

}  // namespace

extern "C" {

int64_t hydro_q_elems(int n_species) { return (int64_t)26 * (6 + n_species) * QCELL; }
int64_t hydro_f_elems(int n_species) { return (int64_t)3 * (6 + n_species) * NFACE; }
int64_t hydro_workspace_bytes(void) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int64_t total = 0;
    for (auto &kv : g_ws)
        if (kv.first.first == dev) total += kv.second.bytes;
    if constexpr (NSUB == 16) total += tiled_work_bytes(dev);
    return total;
}
int hydro_subgrid_n(void) { return NSUB; }

const char *hydro_strerror(int code) {
    switch (code) {
    case HYDRO_OK: return "ok";
    case HYDRO_EINVAL: return "invalid argument";
    case HYDRO_ENODEV: return "the current device is not a gfx950 GPU";
    case HYDRO_ESCRATCH:
        return "batch larger than hydro_step_noalloc's scratch (HYDRO_NOALLOC_MAX_SUB subgrids)";
    case HYDRO_ELAUNCH:
        std::snprintf(g_err, sizeof g_err, "HIP error: %s", hipGetErrorString(g_last_hip));
        return g_err;
    default: return "unknown error code";
    }
}

int hydro_reconstruct(const hydro_params *params, const hydro_batch *batch, const double *U,
                      double *Q, const int64_t *q_offset, void *stream) {
    int rc = check_common(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U || !Q || !q_offset || !aligned8(U) || !aligned8(Q)) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_plain_reconstruct(make_args(params, batch), U, Q, q_offset,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_flux(const hydro_params *params, const hydro_batch *batch, const double *Q,
               const int64_t *q_offset, double *F, const int64_t *f_offset, double *amax,
               int32_t *status, void *stream) {
    int rc = check_common(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!Q || !q_offset || !F || !f_offset || !amax || !aligned8(Q) || !aligned8(F))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_plain_flux(make_args(params, batch), Q, q_offset, F, f_offset, amax,
                                     status, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_divergence(const hydro_params *params, const hydro_batch *batch, const double *F,
                     const int64_t *f_offset, const double *U_in, double *U_out, void *stream) {
    int rc = check_common(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!F || !f_offset || !U_in || !U_out || U_in == U_out) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_plain_divergence(make_args(params, batch), F, f_offset, U_in, U_out,
                                           static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_variant_count(void) { return fused_variant_count(); }
const char *hydro_variant_name(int variant) { return fused_variant_name(variant); }

int hydro_step_variant(const hydro_params *params, const hydro_batch *batch, const double *U_in,
                       double *U_out, double *amax, int32_t *status, int variant, void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (variant < 0 || variant >= fused_variant_count()) return HYDRO_EINVAL;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U_in || !U_out || !amax || U_in == U_out || !aligned8(U_in) || !aligned8(U_out))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    return launch_step(make_args(params, batch), U_in, U_out, amax, status, variant, stream);
}

int hydro_selected_variant(int n_sub, int max_species) {
    (void)max_species;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load_locked();
        auto it = g_tuned.find(bucket_of(n_sub));
        if (it != g_tuned.end()) return it->second;
    }
    return fused_default_variant(n_sub);
}

int hydro_step(const hydro_params *params, const hydro_batch *batch, const double *U_in,
               double *U_out, double *amax, int32_t *status, void *stream) {
    if (!batch) return HYDRO_EINVAL;
    if constexpr (NSUB == 16) {
        // the eight 8^3 tiles of every subgrid through the 8^3 fused kernel
        int rc = check_common(params, batch);
        if (rc) return rc;
        if (batch->n_sub == 0) return HYDRO_OK;
        if (!U_in || !U_out || !amax || U_in == U_out || !aligned8(U_in) || !aligned8(U_out))
            return HYDRO_EINVAL;
        if ((rc = check_device())) return rc;
        hipError_t e = launch_tiled_step(make_args(params, batch), U_in, U_out, amax, status,
                                         stream);
        return e == hipSuccess ? HYDRO_OK : fail_hip(e);
    } else {
        return hydro_step_variant(params, batch, U_in, U_out, amax, status,
                                  hydro_selected_variant(batch->n_sub, 5), stream);
    }
}

int hydro_step_noalloc(const hydro_params *params, const hydro_batch *batch,
                       const double *U_in, double *U_out, double *amax, int32_t *status,
                       void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub > HYDRO_NOALLOC_MAX_SUB) return HYDRO_ESCRATCH;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U_in || !U_out || !amax || U_in == U_out || !aligned8(U_in) || !aligned8(U_out))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    const int variant = hydro_selected_variant(batch->n_sub, 5);
    StepArgs a = make_args(params, batch);
    if (fused_needs_scratch(a, variant)) {
        if ((rc = noalloc_scratch(&a.scratch))) return rc;
        // the words this launch uses start at zero, whatever an earlier call
        // left behind
        const int64_t words = fused_scratch_bytes(batch->n_sub) / 4;
        hipStream_t st = static_cast<hipStream_t>(stream);
        hipLaunchKernelGGL(k_clear_words, dim3((unsigned)((words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024)),
                           dim3(256), 0, st, a.scratch, words);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail_hip(e);
    }
    return launch_step(a, U_in, U_out, amax, status, variant, stream);
}

int hydro_step_io(const hydro_params *params, const hydro_batch *batch,
                  const int64_t *out_offset, const double *U_in, double *U_out,
                  double *amax, int32_t *status, void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!out_offset || !U_in || !U_out || !amax || !aligned8(U_in) || !aligned8(U_out))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    StepArgs a = make_args(params, batch);
    a.out_offset = out_offset;
    return launch_step(a, U_in, U_out, amax, status, hydro_selected_variant(batch->n_sub, 5),
                       stream);
}

int hydro_step_gather(const hydro_params *params, const hydro_batch *batch,
                      const hydro_ghost_map *map, const double *U_in, double *U_out,
                      double *amax, int32_t *status, void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!map || !map->src || !map->mode || !U_in || !U_out || !amax || U_in == U_out ||
        !aligned8(U_in) || !aligned8(U_out))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    StepArgs a = make_args(params, batch);
    a.gsrc = map->src;
    a.gmode = map->mode;
    return launch_step(a, U_in, U_out, amax, status, hydro_selected_variant(batch->n_sub, 5),
                       stream);
}

int hydro_autotune(const hydro_params *params, const hydro_batch *batch, const double *U_in,
                   double *U_out, double *amax, int32_t *status, int reps, float *times_ms,
                   void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0 || reps < 1) return HYDRO_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return fail_hip(e);
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        hipEventDestroy(e0);
        return fail_hip(e);
    }
    int best = -1;
    float best_t = 0.f;
    for (int v = 0; v < fused_variant_count() && rc == HYDRO_OK; v++) {
        rc = hydro_step_variant(params, batch, U_in, U_out, amax, status, v, stream);  // warm-up
        if (rc) break;
        hipEventRecord(e0, st);
        for (int r = 0; r < reps && rc == HYDRO_OK; r++)
            rc = hydro_step_variant(params, batch, U_in, U_out, amax, status, v, stream);
        hipEventRecord(e1, st);
        if ((e = hipEventSynchronize(e1)) != hipSuccess) {
            rc = fail_hip(e);
            break;
        }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (times_ms) times_ms[v] = ms;
        if (best < 0 || ms < best_t) {
            best = v;
            best_t = ms;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tuned[bucket_of(batch->n_sub)] = best;
    tune_save_locked();
    return best;
}

int hydro_plan_create(const hydro_params *params, const hydro_batch *batch, const double *U_in,
                      double *U_out, double *amax, int32_t *status, void *stream,
                      hydro_plan **plan_out) {
    (void)stream;
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (!plan_out || batch->n_sub == 0 || !U_in || !U_out || !amax || U_in == U_out)
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hydro_plan *p = new (std::nothrow) hydro_plan();
    if (!p) return HYDRO_EINVAL;
    p->args = make_args(params, batch);
    p->U_in = U_in;
    p->U_out = U_out;
    p->amax = amax;
    p->status = status;
    p->variant = hydro_selected_variant(batch->n_sub, 5);
    apply_variant(p->args, p->variant);
    if ((rc = batch_unpaired(batch, &p->args.unpaired))) {
        delete p;
        return rc;
    }
    if (fused_needs_scratch(p->args, p->variant)) {
        rc = alloc_scratch(fused_scratch_bytes(batch->n_sub), &p->scratch);
        if (rc) {
            delete p;
            return rc;
        }
        p->args.scratch = p->scratch;
    }
    hipError_t e = plan_build(p);
    if (e != hipSuccess) {
        if (p->scratch) hipFree(p->scratch);
        delete p;
        return fail_hip(e);
    }
    *plan_out = p;
    return HYDRO_OK;
}

int hydro_plan_set_dt(hydro_plan *plan, double dt) {
    if (!plan) return HYDRO_EINVAL;
    plan->args.dt = dt;
    hipError_t e = plan_build(plan);
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_plan_launch(hydro_plan *plan, void *stream) {
    if (!plan) return HYDRO_EINVAL;
    hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_plan_destroy(hydro_plan *plan) {
    if (!plan) return HYDRO_EINVAL;
    hipGraphExecDestroy(plan->exec);
    hipGraphDestroy(plan->graph);
    if (plan->scratch) hipFree(plan->scratch);
    delete plan;
    return HYDRO_OK;
}

// ---- device-resident time integration ---------------------------------------

int hydro_fill_ghosts(const hydro_batch *batch, const hydro_ghost_map *map, double *U,
                      int32_t *status, void *stream) {
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!map || !map->src || !map->mode || !U || !aligned8(U)) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_fill_ghosts(batch->n_sub, batch->fstride, batch->offset,
                                      batch->n_species, map->src, map->mode, U, status,
                                      static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_rate(const hydro_params *params, const hydro_batch *batch, const double *U_in,
               double *R, double *amax, int32_t *status, void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U_in || !R || !amax || U_in == R || !aligned8(U_in) || !aligned8(R)) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    StepArgs a = make_args(params, batch);
    a.rate = 1;
    return launch_step(a, U_in, R, amax, status, hydro_selected_variant(batch->n_sub, 5), stream);
}

int hydro_cfl_dt(const hydro_batch *batch, const double *amax, double cfl, double t_end,
                 double *clock, void *stream) {
    int rc = check_batch(batch);
    if (rc) return rc;
    if ((batch->n_sub > 0 && !amax) || !clock || !(cfl > 0.0)) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_cfl_dt(batch->n_sub, batch->h, amax, cfl, t_end, clock,
                                 static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_rk_stage(const hydro_params *params, const hydro_batch *batch, const double *U_in,
                   double *U_out, const double *U0, double a, double b, const double *clock,
                   double *amax, int32_t *status, void *stream) {
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U_in || !U_out || !U0 || !clock || !amax || U_in == U_out || !aligned8(U_in) ||
        !aligned8(U_out) || !aligned8(U0))
        return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    StepArgs sa = make_args(params, batch);
    sa.clock = clock;
    sa.U0 = U0;
    sa.c0 = a;
    sa.c1 = b;
    return launch_step(sa, U_in, U_out, amax, status, hydro_selected_variant(batch->n_sub, 5),
                       stream);
}

int hydro_tau_resync(const hydro_params *params, const hydro_batch *batch, double *U,
                     void *stream) {
    int rc = check_common(params, batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U || !aligned8(U)) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_tau_resync(make_args(params, batch), U, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

int hydro_rk_update(const hydro_batch *batch, double a, const double *U0, double b,
                    const double *Uk, const double *R, const double *clock, double *U_out,
                    void *stream) {
    int rc = check_batch(batch);
    if (rc) return rc;
    if (batch->n_sub == 0) return HYDRO_OK;
    if (!U0 || !Uk || !R || !clock || !U_out) return HYDRO_EINVAL;
    if ((rc = check_device())) return rc;
    hipError_t e = launch_rk_update(batch->n_sub, batch->fstride, batch->offset,
                                    batch->n_species, a, U0, b, Uk, R, clock, U_out,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

namespace {

// One SSP-RK3 step, enqueued on `st` (recorded when st is capturing).  The
// fused stages read their ghost cells through the map (ra.gsrc, ra.gmode), so
// no stage needs a fill pass and the ghost layers of U, U1 and U2 are never
// read.
hipError_t enqueue_rk3_step(const StepArgs &ra, int variant, double *U, double *U1, double *U2,
                            double *R, double *amax, int32_t *status, double *clock, double cfl,
                            double t_end, hipStream_t st) {
    const int n = ra.n_sub, fs = ra.fstride;
    hipError_t e;
    if ((e = launch_fused_step(ra, U, R, amax, status, variant, st))) return e;
    if ((e = launch_cfl_dt(n, ra.h, amax, cfl, t_end, clock, st))) return e;
    if ((e = launch_rk_update(n, fs, ra.offset, ra.n_species, 0.0, U, 1.0, U, R, clock, U1, st)))
        return e;
    StepArgs sa = ra;               // fused stages with dt from the device clock
    sa.rate = 0;
    sa.clock = clock;
    sa.U0 = U;
    sa.c0 = 0.75;
    sa.c1 = 0.25;
    if ((e = launch_fused_step(sa, U1, U2, amax, status, variant, st))) return e;
    sa.c0 = 1.0 / 3.0;
    sa.c1 = 2.0 / 3.0;
    return launch_fused_step(sa, U2, U, amax, status, variant, st);
}

}  // namespace

int hydro_rk3_create(const hydro_params *params, const hydro_batch *batch,
                     const hydro_ghost_map *map, double *U, double *U1, double *U2, double *R,
                     double *amax, int32_t *status, double *clock, double cfl, double t_end,
                     void *stream, hydro_rk3 **plan_out) {
    (void)stream;
    int rc = check_fused(params, batch);
    if (rc) return rc;
    if (!plan_out || batch->n_sub == 0 || !map || !map->src || !map->mode || !U || !U1 || !U2 ||
        !R || !amax || !clock || !(cfl > 0.0))
        return HYDRO_EINVAL;
    const double *bufs[4] = {U, U1, U2, R};
    for (int i = 0; i < 4; i++) {
        if (!aligned8(bufs[i])) return HYDRO_EINVAL;
        for (int j = 0; j < i; j++)
            if (bufs[i] == bufs[j]) return HYDRO_EINVAL;
    }
    if ((rc = check_device())) return rc;
    StepArgs ra = make_args(params, batch);
    ra.rate = 1;
    ra.gsrc = map->src;
    ra.gmode = map->mode;
    const int variant = hydro_selected_variant(batch->n_sub, 5);
    if ((rc = batch_unpaired(batch, &ra.unpaired))) return rc;
    hydro_rk3 *p = new (std::nothrow) hydro_rk3();
    if (!p) return HYDRO_EINVAL;
    if (fused_needs_scratch(ra, variant)) {
        // allocated before the capture (no allocation may be captured); the
        // stages run one after another, so they share it
        rc = alloc_scratch(fused_scratch_bytes(batch->n_sub), &p->scratch);
        if (rc) {
            delete p;
            return rc;
        }
        ra.scratch = p->scratch;
    }
    hipStream_t cs;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (p->scratch) hipFree(p->scratch);
        delete p;
        return fail_hip(e);
    }
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = enqueue_rk3_step(ra, variant, U, U1, U2, R, amax, status, clock, cfl,
                                         t_end, cs);
        e = hipStreamEndCapture(cs, &p->graph);
        if (e1 != hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (p->graph) hipGraphDestroy(p->graph);
        if (p->scratch) hipFree(p->scratch);
        delete p;
        return fail_hip(e);
    }
    *plan_out = p;
    return HYDRO_OK;
}

int hydro_rk3_launch(hydro_rk3 *plan, int n_steps, void *stream) {
    if (!plan || n_steps < 0) return HYDRO_EINVAL;
    for (int i = 0; i < n_steps; i++) {
        hipError_t e = hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) return fail_hip(e);
    }
    return HYDRO_OK;
}

int hydro_rk3_destroy(hydro_rk3 *plan) {
    if (!plan) return HYDRO_EINVAL;
    hipGraphExecDestroy(plan->exec);
    hipGraphDestroy(plan->graph);
    if (plan->scratch) hipFree(plan->scratch);
    delete plan;
    return HYDRO_OK;
}

int hydro_copy_blocks(const double *src, int64_t src_rows, const int64_t *src_row, double *dst,
                      int64_t dst_rows, const int64_t *dst_row0, const int64_t *dst_row1, int n,
                      int64_t row_elems, void *stream) {
    if (n < 0 || row_elems < 1 || src_rows < 0 || dst_rows < 0) return HYDRO_EINVAL;
    if (n == 0) return HYDRO_OK;
    if (!src || !dst || !src_row || !dst_row0) return HYDRO_EINVAL;
    const int64_t chunks = (row_elems + kCopyChunk - 1) / kCopyChunk;
    if ((int64_t)n * chunks > INT32_MAX) return HYDRO_EINVAL;
    int rc = check_device();
    if (rc) return rc;
    const int vec2 = row_elems % 2 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(dst) % 16 == 0;
    hipLaunchKernelGGL(k_copy_blocks, dim3((unsigned)(n * chunks)), dim3(kCopyThreads), 0,
                       static_cast<hipStream_t>(stream), src, src_rows, src_row, dst, dst_rows,
                       dst_row0, dst_row1, row_elems, (int)chunks, vec2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? HYDRO_OK : fail_hip(e);
}

}  // extern "C"
