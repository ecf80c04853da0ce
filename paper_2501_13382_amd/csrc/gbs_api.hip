// Host side of libgbs: C ABI, argument validation, planning (receiver
// ordering, passes over the table, culled work lists), launches, graphs and
// the autotuner.  See include/gbs.h for the contract of every entry point.
#include "gbs.h"
#include "gbs_internal.h"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

// kernels (gbs_kernels.hip)
namespace gbs {
__global__ void k_fill_f64(double*, int64_t, double);
__global__ void k_fill_i32(int32_t*, int64_t, int32_t);
__global__ void k_reset_counter(unsigned*);
__global__ void k_bbox_partial(const double*, int64_t, double*);
__global__ void k_bbox_final(const double*, int, double*);
__global__ void k_morton(const double*, int64_t, const double*, uint32_t*, int32_t*);
__global__ void k_gather_rcv(const double*, int64_t, int64_t, const int32_t*, double*, double*, double*, double*,
                             int32_t*, int*);
__global__ void k_patches(const double*, const double*, const double*, int64_t, int64_t, int, Patch*);
__global__ void k_sphere_of_spheres(const Patch*, int, int, int, Patch*);
__global__ void k_src_ranges(const int64_t*, const int32_t*, int64_t, int32_t, int64_t, const int64_t*, int, int32_t,
                             int64_t*, int*);
__global__ void k_job_consts(const double*, const double*, const double*, const double*, int32_t, int32_t, double,
                             double, const int64_t*, int64_t, int64_t, JobConst*, int*);
__global__ void k_make_splits(const int64_t*, int32_t, int64_t, int64_t, int64_t, int32_t, int64_t, CullSplit*,
                              int32_t*, int64_t*);
__global__ void k_seg2ray(const int64_t*, int64_t, int64_t, int64_t, int32_t*);
__global__ void k_records(int64_t, const double*, const double*, const double*, const double*, const double*,
                          const int64_t*, int64_t, const int32_t*, int32_t, const double*, const double*,
                          const int32_t*, int64_t, const int64_t*, int64_t, SegRec*, int*, unsigned long long*);
template <bool FILL, int NB>
__global__ void k_cull(const JobConst*, const SegRec*, const Patch*, const Patch*, int, int, const int64_t*,
                       const CullSplit*,
                       const int32_t*, const unsigned long long*, int, int, int32_t*, const int64_t*, int32_t*,
                       unsigned char*, unsigned*, int64_t, int32_t*, const int32_t*);
__global__ void k_cull_need(const unsigned*, unsigned*);
template <bool SCATTER>
__global__ void k_cull_order(const unsigned*, int, int, int, int64_t, unsigned*, int32_t*);
template <int NB>
__global__ void k_cull_replay(const CullSplit*, int, int, int, const int64_t*, const int64_t*, const unsigned char*,
                              const unsigned*, int64_t, const int32_t*, int32_t*);
size_t cull_batch_bytes(int nb);
int cull_batch_regions();
int cull_batch_ctr_stride();
int cull_batch_block();
template <int NB>
__global__ void k_cull_hyper(const JobConst*, const SegRec*, const Patch*, int, int, int, const CullSplit*,
                             const int32_t*, unsigned long long*, const Patch*, int, int, unsigned*);
__global__ void k_item_lengths(const int64_t*, int32_t, int, int, const int64_t*, int32_t*);
__global__ void k_iota(int32_t*, int32_t);
__global__ void k_seg_keys(int64_t, const SegRec*, const JobConst*, int32_t, int32_t, const double*,
                           unsigned long long*, int32_t*);
__global__ void k_permute_rec(int64_t, const SegRec*, const int32_t*, SegRec*);
__global__ void k_frames(int64_t, const double*, const double*, const double*, const double*, FrameRec*, int*);
__global__ void k_permute_frames(int64_t, const FrameRec*, const int32_t*, FrameRec*);
template <int MODE, int NR, bool COUNT>
__global__ void k_pairs(const JobConst*, const Work*, const int32_t*, int32_t, unsigned*, const int32_t*,
                        const SegRec*, const FrameRec*, const double*, const double*, const double*, const double*,
                        double*, unsigned long long*);
__global__ void k_work_counts(const int32_t*, const int32_t*, int32_t, int32_t, int32_t*);
__global__ void k_make_work(const int32_t*, const int64_t*, int, int, const int64_t*, const int32_t*, int32_t, int32_t,
                            Work*, int32_t*, int32_t*, int32_t*);
__global__ void k_reduce_partials(const JobConst*, const int32_t*, const int32_t*, int32_t, int32_t, int,
                                  const int32_t*, int64_t, const double*, double*, double*, int);
__global__ void k_tl(const double*, int64_t, double*);
template <int MODE>
__global__ void k_adjoint(const JobConst*, const Work*, const int32_t*, int32_t, unsigned*, const int32_t*,
                          const SegRec*, const FrameRec*, const double*, const double*, const double*, const double*,
                          const int32_t*, int64_t, const double*, double*, const int32_t*, Fixed*, const double*,
                          double*, double*);
__global__ void k_reduce_adjoint(const JobConst*, const int32_t*, const int32_t*, int32_t, int32_t, const int32_t*,
                                 int64_t, const double*, double*);
__global__ void k_sum_jobs(const double*, int32_t, int64_t, double*);
__global__ void k_face_scatter(int64_t, const int64_t*, int64_t, const int32_t*, int32_t, const double*,
                               const double*, const int32_t*, const Fixed*, const double*, Fixed*);
__global__ void k_dgamma(const double*, int32_t, double*);
__global__ void k_lambda_l1(const double*, int64_t, double*, int*);
__global__ void k_lambda_l1_sum(const double*, int32_t, int, double*);
__global__ void k_fixed_scales(const JobConst*, const double*, int32_t, int64_t, const unsigned long long*, double*);
__global__ void k_reduce_eps(const int32_t*, const int32_t*, int32_t, const double*, double*);
__global__ void k_fixed_flush(const Fixed*, int64_t, const double*, double*);
// ray tracing (gbs_trace.hip)
template <bool COUNT>
__global__ void k_trace(int64_t, int, const double*, const int32_t*, const double*, const double*, const double*,
                        const double*,
                        const int32_t*, int, int, int, double, int, int64_t*, int*, const int64_t*, const int64_t*,
                        double*, double*, double*, double*, double*, int64_t*, int32_t*, const double*, double*);
__global__ void k_trace_face_counts(int64_t, const int64_t*, int64_t*);
// broadband synthesis (gbs_ir.hip)
__global__ void k_ir_twiddles(int, double2*);
__global__ void k_ir_scatter(const double*, int, int, int64_t, int, const double*, int, int, double2*);
__global__ void k_ir_fft(const double2*, int, int, const double2*, double, int, double*);
__global__ void k_trace_close(const int64_t*, int64_t, int64_t, int64_t*);
}  // namespace gbs

using namespace gbs;

// Scratch of the allocation-free forward (gbs_forward_noalloc): one array per
// device, loaded with the code object and held until the process ends.  In
// host code `scratch` names a host-side stand-in, not device memory: the
// device address comes from hipGetSymbolAddress, once per device, at
// gbs_create (scratch_base()), and only that address is ever passed on.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

struct GbsError : std::runtime_error {
    int code;
    GbsError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define GBS_HIP(call)                                                                                     \
    do {                                                                                                  \
        hipError_t e_ = (call);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            throw GbsError(e_ == hipErrorOutOfMemory ? GBS_E_OOM : GBS_E_HIP,                             \
                           std::string(#call) + ": " + hipGetErrorString(e_));                            \
    } while (0)

#define GBS_CHECK(cond, msg)                                   \
    do {                                                       \
        if (!(cond)) throw GbsError(GBS_E_INVALID, (msg));     \
    } while (0)

// Device address of `scratch` on each device, looked up once per device with
// that device current (gbs_create); null until then.
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_base;

void scratch_init(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_base.size() <= device) g_scratch_base.resize(device + 1, nullptr);
    if (g_scratch_base[device]) return;
    void* p = nullptr;
    GBS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    GBS_CHECK(p != nullptr, "static scratch has no device address");
    g_scratch_base[device] = p;
}

void* scratch_base(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= (int)g_scratch_base.size() || !g_scratch_base[device])
        throw GbsError(GBS_E_STATE, "static scratch not set up on this device");
    return g_scratch_base[device];
}

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads); }

// Device fill with a kernel (no memset nodes, so it is safe in captured graphs).
void fill(hipStream_t st, double* p, int64_t n, double v) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>(4096, blocks_for(n, 256))), dim3(256), 0, st, p,
                       n, v);
}

// Grow-only device buffers, keyed by name.  In arena mode (the
// allocation-free forward) every buffer is carved from one fixed device
// region instead: nothing is allocated or freed, and a call that needs more
// than the region fails with GBS_E_UNSUPPORTED.
// Work-unit size of calls that run in several passes (smaller than
// kWorkChunk: a short pass cannot hide a long last unit).
constexpr int kWorkChunkPasses = 512;

struct Workspace {
    std::map<std::string, std::pair<void*, size_t>> bufs;
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;    // also drained before a buffer is freed
    hipStream_t pair_streams[2] = {nullptr, nullptr};   // likewise
    bool frozen = false;                  // set during graph capture: no allocation allowed
    char* arena = nullptr;                // arena mode: base of the region, its size, bytes handed out
    size_t arena_cap = 0, arena_used = 0;
    Workspace() = default;
    Workspace(void* base, size_t cap) : arena(static_cast<char*>(base)), arena_cap(cap) {}
    ~Workspace() { release(); }
    // Device bytes this workspace holds (arena mode: handed out this call).
    size_t held() const {
        if (arena) return arena_used;
        size_t n = 0;
        for (const auto& kv : bufs) n += kv.second.second;
        return n;
    }
    void release() {
        if (!arena)
            for (auto& kv : bufs)
                if (kv.second.first) (void)hipFree(kv.second.first);
        bufs.clear();
    }
    template <typename T>
    T* get(const std::string& name, size_t count) {
        size_t bytes = std::max<size_t>(count * sizeof(T), 256);
        auto& b = bufs[name];
        if (arena) {
            if (b.second < bytes) {   // a new slice; a smaller earlier one of the same name is left unused
                const size_t off = (arena_used + 255) & ~size_t(255);
                if (off > arena_cap || bytes > arena_cap - off)
                    throw GbsError(GBS_E_UNSUPPORTED,
                                   "gbs_forward_noalloc: the call needs more than the " +
                                       std::to_string(arena_cap >> 20) + " MiB of static scratch (buffer '" + name +
                                       "' of " + std::to_string(bytes) + " bytes at offset " + std::to_string(off) +
                                       "); use gbs_forward");
                b.first = arena + off;
                b.second = bytes;
                arena_used = off + bytes;
            }
            return static_cast<T*>(b.first);
        }
        if (b.second < bytes) {
            GBS_CHECK(!frozen, "internal: workspace growth during graph capture");
            if (b.first) {
                GBS_HIP(hipStreamSynchronize(stream));
                if (copy_stream) GBS_HIP(hipStreamSynchronize(copy_stream));
                for (hipStream_t ps : pair_streams)
                    if (ps) GBS_HIP(hipStreamSynchronize(ps));
                GBS_HIP(hipFree(b.first));
                b.first = nullptr;
                b.second = 0;
            }
            size_t cap = bytes + bytes / 4;
            GBS_HIP(hipMalloc(&b.first, cap));
            b.second = cap;
        }
        return static_cast<T*>(b.first);
    }
};

struct RcvPlan {
    int64_t n = 0, n_pad = 0;
    int per = 0;                 // receivers per patch
    int n_patch = 0, n_super = 0, n_hyper = 0;
    double *rx = nullptr, *ry = nullptr, *rz = nullptr, *r2 = nullptr;
    int32_t* perm = nullptr;
    Patch* patches = nullptr;
    Patch* supers = nullptr;
    Patch* hypers = nullptr;      // groups of kHyperSupers super-patches
    const double* bbox = nullptr; // receivers' bounding box (min xyz, max xyz)
};

struct PassRange {
    int64_t ray_begin, ray_end, seg_begin, seg_end, face_begin, face_end;
};

}  // namespace

struct gbs_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 0;
    std::string err;
    gbs_stats stats{};
    std::unique_ptr<Workspace> ws{new Workspace};
    int tuned_nr[3] = {0, 0, 0};      // per mode, 0 = not tuned
    int tuned_chunk[3] = {0, 0, 0};
    // streaming of host-resident tables: pass i+1 is copied on copy_stream
    // while pass i computes; two staging slots, ordered by these events
    hipStream_t copy_stream = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t released[2] = {nullptr, nullptr};
    // calls in several passes: the pair kernel of pass i runs on
    // pair_stream[i % 2] (ready: its lists are laid out; done: its partial
    // sums are written), so that it overlaps the end of pass i - 1's
    hipStream_t pair_stream[2] = {nullptr, nullptr};
    hipEvent_t pair_ready[2] = {nullptr, nullptr};
    hipEvent_t pair_done[2] = {nullptr, nullptr};
    // list-length reads of up to two planned passes: pinned host words (list
    // total, status word) per slot and the events behind their copies; made
    // at creation so that no call allocates them
    int64_t* plan_words = nullptr;    // [2][3]: total, status, cull batches
    hipEvent_t planned[2] = {nullptr, nullptr};
    // the most batch records one region of the cull has needed in a pass:
    // sizes the regions of later passes
    int64_t cull_region_need = 0;
    // the last gbs_trace_count: its token, what it counted, and its sizes
    // (the per-ray offsets stay in the workspace for gbs_trace to reuse)
    int64_t trace_token = 0, trace_token_next = 0;
    std::vector<uint64_t> trace_sig;
    int64_t trace_tot[2] = {0, 0};
    int trace_groups = 0;
};

struct gbs_graph {
    gbs_ctx* ctx = nullptr;
    std::unique_ptr<Workspace> ws{new Workspace};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

void set_err(gbs_ctx* ctx, const std::string& m) {
    if (ctx) ctx->err = m;
}

template <typename F>
int guarded(gbs_ctx* ctx, F&& f) {
    try {
        int rc = f();
        if (rc == GBS_OK && ctx) ctx->err.clear();
        return rc;
    } catch (const GbsError& e) {
        set_err(ctx, e.what());
        return e.code;
    } catch (const std::bad_alloc&) {
        set_err(ctx, "host allocation failed");
        return GBS_E_OOM;
    } catch (const std::exception& e) {
        set_err(ctx, e.what());
        return GBS_E_HIP;
    } catch (...) {
        set_err(ctx, "unknown failure");
        return GBS_E_HIP;
    }
}

// ------------------------------------------------------------- validation
struct Args {
    const gbs_rays* rays;
    const gbs_segs* segs;
    const gbs_faces* faces;
    const double* rcv;
    int64_t n_rcv;
    const double* freqs;
    int32_t n_freq;
    const double* eps;
    const gbs_params* params;
};

void validate_host(const Args& a) {
    GBS_CHECK(a.rays && a.segs && a.faces && a.params, "null struct argument");
    const gbs_params& p = *a.params;
    GBS_CHECK(std::isfinite(p.c) && p.c > 0, "params.c must be finite and > 0");
    GBS_CHECK(std::isfinite(p.gate_G) && p.gate_G > 0, "params.gate_G must be finite and > 0");
    GBS_CHECK(p.mode == GBS_MODE_F64 || p.mode == GBS_MODE_MIX || p.mode == GBS_MODE_F32, "params.mode invalid");
    GBS_CHECK((p.flags & ~(GBS_FLAG_TABLE_HOST | GBS_FLAG_VALIDATE | GBS_FLAG_COUNT_ACTIVE |
                            GBS_FLAG_TIME_KERNELS)) == 0,
              "params.flags has unknown bits");
    GBS_CHECK(p.chunk_segs >= 0, "params.chunk_segs must be >= 0");
    GBS_CHECK(p.rcv_per_lane == 0 || p.rcv_per_lane == 1 || p.rcv_per_lane == 2 || p.rcv_per_lane == 4,
              "params.rcv_per_lane must be 0, 1, 2 or 4");
    GBS_CHECK(p.work_chunk == 0 || (p.work_chunk >= 256 && p.work_chunk <= 65536 &&
                                    (p.work_chunk & (p.work_chunk - 1)) == 0),
              "params.work_chunk must be 0 or a power of two in [256, 65536]");
    GBS_CHECK(a.rays->n_src >= 0 && a.rays->n_rays >= 0 && a.segs->n_segs >= 0 && a.n_rcv >= 0 && a.n_freq >= 0,
              "negative size");
    GBS_CHECK(a.faces->n_faces >= 0, "negative face count");
    if (a.n_freq > kMaxBands)
        throw GbsError(GBS_E_UNSUPPORTED, "at most 64 bands per call");
    GBS_CHECK(a.n_rcv <= (int64_t)INT32_MAX - 4096, "too many receivers");
    GBS_CHECK(a.segs->n_segs <= (int64_t)INT32_MAX, "too many segments");
    GBS_CHECK(a.rays->n_rays == 0 || a.rays->n_src > 0, "rays without sources");
    if (a.rays->n_rays > 0)
        GBS_CHECK(a.rays->ray_ptr && a.rays->ray_w && a.rays->ray_src, "null ray array");
    if (a.rays->n_rays == 0) GBS_CHECK(a.segs->n_segs == 0, "segments without rays");
    GBS_CHECK(a.rays->ray_ptr || a.rays->n_rays == 0, "null ray_ptr");
    if (a.segs->n_segs > 0)
        GBS_CHECK(a.segs->a && a.segs->t && a.segs->s0 && a.segs->lo && a.segs->hi && a.segs->face_ptr,
                  "null segment array");
    if (a.faces->n_faces > 0) GBS_CHECK(a.faces->gamma, "null gamma");
    if (a.n_rcv > 0) GBS_CHECK(a.rcv, "null receivers");
    if (a.n_freq > 0) GBS_CHECK(a.freqs && a.eps, "null freqs/eps");
}

// The device status word (StatusBit) as an error.
void check_status(int bits) {
    if (bits == 0) return;
    std::string m = "invalid input:";
    if (bits & kBadSegment)
        m += " segment values (non-finite a, s0, lo or hi, lo > hi, |t| != 1, or a frame vector e1 not unit or not "
             "normal to t);";
    if (bits & kBadFacePtr) m += " face_ptr (not a non-decreasing CSR from 0);";
    if (bits & kBadFaceId) m += " face id outside [0, n_faces);";
    if (bits & kBadRayPtr) m += " ray_ptr (not a non-decreasing CSR from 0 to n_segs);";
    if (bits & kBadRayWeight) m += " ray weight (non-finite or negative);";
    if (bits & kBadReceiver) m += " receiver coordinate (non-finite);";
    if (bits & kBadRaySource) m += " ray_src (outside [0, n_src) or not non-decreasing);";
    if (bits & kBadLambda) m += " lambda (non-finite);";
    if (bits & kBadJob) m += " frequency, eps, alpha or eps_e2 (non-finite, or not > 0; alpha >= 0);";
    throw GbsError(GBS_E_INVALID, m);
}

// ------------------------------------------------------------- planning
struct Planner {
    gbs_ctx* ctx;
    Workspace& ws;
    hipStream_t st;
    const Args& a;
    int mode, nr;
    int n_jobs;
    const int64_t* d_src_off = nullptr;   // device: first segment of each source, [n_src + 1]
    std::vector<int64_t> h_src_off;       // host tables: the same, computed on the host and copied
    std::vector<PassRange> passes;
    std::vector<int64_t> h_ray_ptr, h_face_ptr;  // host copies (only when chunking)
    RcvPlan R;
    int* status = nullptr;            // device StatusBit word of this call

    Planner(gbs_ctx* c, Workspace& w, const Args& args, int nr_)
        : ctx(c), ws(w), st(c->stream), a(args), mode(args.params->mode), nr(nr_) {
        ws.stream = st;
        n_jobs = a.rays->n_src * a.n_freq;
    }

    bool table_host() const { return (a.params->flags & GBS_FLAG_TABLE_HOST) != 0; }

    // Clears the status word; the kernels that read the inputs set its bits.
    void reset_status() {
        status = ws.get<int>("status", 2);
        fill(st, reinterpret_cast<double*>(status), 1, 0.0);
    }
    int chunk_override = 0;   // autotuner candidate
    std::string tag;          // graph creation: per-pass names for the buffers the replays read
    // Segments per work unit: the caller's, the tuned one, else kWorkChunk
    // for one pass and kWorkChunkPasses when the call runs in several passes
    // (each pass's pair launch ends on its own longest unit).
    int work_chunk() const {
        if (chunk_override) return chunk_override;
        if (a.params->work_chunk) return a.params->work_chunk;
        if (ctx->tuned_chunk[a.params->mode]) return ctx->tuned_chunk[a.params->mode];
        return passes.size() > 1 ? kWorkChunkPasses : kWorkChunk;
    }

    bool aniso() const { return a.params->eps_e2 != nullptr; }

    // The job inputs checked on the host, for calls with no device work (with
    // work, k_job_consts checks them on the device).  Synchronises.
    void check_jobs_on_host() {
        if (n_jobs == 0) return;
        std::vector<double> f(a.n_freq), e(n_jobs), al(a.params->alpha ? n_jobs : 0), e2(a.params->eps_e2 ? n_jobs : 0);
        GBS_HIP(hipMemcpyAsync(f.data(), a.freqs, sizeof(double) * f.size(), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipMemcpyAsync(e.data(), a.eps, sizeof(double) * e.size(), hipMemcpyDeviceToHost, st));
        if (!al.empty())
            GBS_HIP(hipMemcpyAsync(al.data(), a.params->alpha, sizeof(double) * al.size(), hipMemcpyDeviceToHost, st));
        if (!e2.empty())
            GBS_HIP(hipMemcpyAsync(e2.data(), a.params->eps_e2, sizeof(double) * e2.size(), hipMemcpyDeviceToHost,
                                   st));
        GBS_HIP(hipStreamSynchronize(st));
        int bad = 0;
        for (double x : f) bad |= !(std::isfinite(x) && x > 0);
        for (double x : e) bad |= !(std::isfinite(x) && x > 0);
        for (double x : al) bad |= !(std::isfinite(x) && x >= 0);
        for (double x : e2) bad |= !(std::isfinite(x) && x > 0);
        check_status(bad ? kBadJob : 0);
    }

    // The pair kernel's absorption variant runs whenever absorption is given
    // (a zero alpha then gives bitwise the same sum as none).
    bool absorb() const { return a.params->alpha != nullptr; }

    // First segment of every source (device array d_src_off), and the checks
    // of the ray and face CSR arrays: on the host for host tables, by
    // k_src_ranges otherwise (flags read at the list-length synchronisation,
    // before any beam is evaluated).  No synchronisation for device tables.
    void source_offsets() {
        const int32_t n_src = a.rays->n_src;
        const int64_t n_rays = a.rays->n_rays, n_segs = a.segs->n_segs;
        int64_t* d_off = ws.get<int64_t>("src_off", n_src + 2);
        d_src_off = d_off;
        if (table_host()) {
            std::vector<int64_t>& src_off = h_src_off;
            src_off.assign(n_src + 1, 0);
            const int64_t* rp = a.rays->ray_ptr;
            const int32_t* rs = a.rays->ray_src;
            const int64_t* fp = a.segs->face_ptr;
            GBS_CHECK(rp[0] == 0 && rp[n_rays] == n_segs, "ray_ptr must span the segments");
            // the checks as branch-free reductions over the arrays (they vectorise), then the offsets
            bool src_ok = true, sorted = true, rp_ok = true, fp_ok = true;
            for (int64_t i = 0; i < n_rays; ++i) src_ok &= rs[i] >= 0 && rs[i] < n_src;
            for (int64_t i = 1; i < n_rays; ++i) sorted &= rs[i] >= rs[i - 1];
            for (int64_t i = 0; i < n_rays; ++i) rp_ok &= rp[i + 1] >= rp[i];
            GBS_CHECK(src_ok, "ray_src out of range");
            GBS_CHECK(sorted, "rays must be sorted by source");
            GBS_CHECK(rp_ok, "ray_ptr must be non-decreasing");
            for (int64_t i = 0; i <= n_rays; ++i) {
                const int32_t prev = i == 0 ? -1 : rs[i - 1];
                const int32_t cur = i == n_rays ? n_src : rs[i];
                for (int32_t s = prev + 1; s <= cur; ++s) src_off[s] = rp[i];
            }
            GBS_CHECK(fp[0] == 0, "face_ptr[0] must be 0");
            for (int64_t j = 0; j < n_segs; ++j) fp_ok &= fp[j + 1] >= fp[j];
            GBS_CHECK(fp_ok, "face_ptr must be non-decreasing");
            GBS_CHECK(fp[n_segs] == 0 || a.segs->face_ids, "null face_ids");
            GBS_CHECK(fp[n_segs] == 0 || a.faces->n_faces > 0, "face histories need n_faces > 0");
            GBS_HIP(hipMemcpyAsync(d_off, src_off.data(), sizeof(int64_t) * (n_src + 1), hipMemcpyHostToDevice, st));
        } else {
            hipLaunchKernelGGL(k_src_ranges, dim3(blocks_for(n_rays + 1, 256)), dim3(256), 0, st, a.rays->ray_ptr,
                               a.rays->ray_src, n_rays, n_src, n_segs, a.segs->face_ptr,
                               a.segs->face_ids != nullptr ? 1 : 0, a.faces->n_faces, d_off, status);
            GBS_HIP(hipGetLastError());
        }
    }

    void make_passes() {
        const int64_t n_rays = a.rays->n_rays, n_segs = a.segs->n_segs;
        const int64_t cs = a.params->chunk_segs;
        passes.clear();
        if (n_rays == 0) return;
        bool chunk = table_host() || (cs > 0 && cs < n_segs);
        if (!chunk) {
            passes.push_back({0, n_rays, 0, n_segs, 0, 0});
            return;
        }
        const int64_t* rp;
        const int64_t* fp;
        if (table_host()) {
            rp = a.rays->ray_ptr;
            fp = a.segs->face_ptr;
        } else {
            h_ray_ptr.resize(n_rays + 1);
            h_face_ptr.resize(n_segs + 1);
            GBS_HIP(hipMemcpyAsync(h_ray_ptr.data(), a.rays->ray_ptr, sizeof(int64_t) * (n_rays + 1),
                                   hipMemcpyDeviceToHost, st));
            GBS_HIP(hipMemcpyAsync(h_face_ptr.data(), a.segs->face_ptr, sizeof(int64_t) * (n_segs + 1),
                                   hipMemcpyDeviceToHost, st));
            GBS_HIP(hipStreamSynchronize(st));
            rp = h_ray_ptr.data();
            fp = h_face_ptr.data();
            // the pass ranges come from these arrays: check them before using them
            GBS_CHECK(rp[0] == 0 && rp[n_rays] == n_segs, "ray_ptr must span the segments");
            for (int64_t i = 0; i < n_rays; ++i) GBS_CHECK(rp[i + 1] >= rp[i], "ray_ptr must be non-decreasing");
            GBS_CHECK(fp[0] == 0, "face_ptr[0] must be 0");
            for (int64_t j = 0; j < n_segs; ++j) GBS_CHECK(fp[j + 1] >= fp[j], "face_ptr must be non-decreasing");
        }
        const int64_t limit = cs > 0 ? cs : n_segs;
        int64_t r0 = 0;
        while (r0 < n_rays) {
            int64_t r1 = r0 + 1;
            while (r1 < n_rays && rp[r1 + 1] - rp[r0] <= limit) ++r1;
            passes.push_back({r0, r1, rp[r0], rp[r1], fp[rp[r0]], fp[rp[r1]]});
            r0 = r1;
        }
    }

    // Receivers in Morton order, padded to whole patches; patch and
    // super-patch bounding spheres.
    void plan_receivers(int per) {
        R = RcvPlan{};
        R.n = a.n_rcv;
        R.per = per;
        if (R.n == 0) return;
        R.n_patch = (int)((R.n + per - 1) / per);
        R.n_pad = (int64_t)R.n_patch * per;
        R.n_super = (R.n_patch + kSuperPatches - 1) / kSuperPatches;
        R.n_hyper = (R.n_super + kHyperSupers - 1) / kHyperSupers;
        const int nb = (int)std::min<int64_t>(1024, blocks_for(R.n, 256));
        double* part = ws.get<double>("bbox_part", 6 * nb);
        double* bbox = ws.get<double>("bbox", 6);
        hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, st, a.rcv, R.n, part);
        hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(256), 0, st, part, nb, bbox);
        R.bbox = bbox;
        uint32_t* keys = ws.get<uint32_t>("mkeys", R.n);
        uint32_t* keys2 = ws.get<uint32_t>("mkeys2", R.n);
        int32_t* vals = ws.get<int32_t>("mvals", R.n);
        int32_t* vals2 = ws.get<int32_t>("mvals2", R.n);
        hipLaunchKernelGGL(k_morton, dim3(blocks_for(R.n, 256)), dim3(256), 0, st, a.rcv, R.n, bbox, keys, vals);
        size_t tmp = 0;
        GBS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, keys, keys2, vals, vals2, (int)R.n, 0, 30, st));
        void* t = ws.get<char>("cub_tmp_sort", tmp);
        GBS_HIP(hipcub::DeviceRadixSort::SortPairs(t, tmp, keys, keys2, vals, vals2, (int)R.n, 0, 30, st));
        R.rx = ws.get<double>("rx", R.n_pad);
        R.ry = ws.get<double>("ry", R.n_pad);
        R.rz = ws.get<double>("rz", R.n_pad);
        R.r2 = ws.get<double>("r2", R.n_pad);
        R.perm = ws.get<int32_t>("perm", R.n_pad);
        hipLaunchKernelGGL(k_gather_rcv, dim3(blocks_for(R.n_pad, 256)), dim3(256), 0, st, a.rcv, R.n, R.n_pad,
                           vals2, R.rx, R.ry, R.rz, R.r2, R.perm, status);
        R.patches = ws.get<Patch>("patches", R.n_patch);
        R.supers = ws.get<Patch>("supers", R.n_super);
        hipLaunchKernelGGL(k_patches, dim3(R.n_patch), dim3(64), 0, st, R.rx, R.ry, R.rz, R.n_pad, (int64_t)per,
                           R.n_patch, R.patches);
        hipLaunchKernelGGL(k_sphere_of_spheres, dim3(R.n_super), dim3(64), 0, st, R.patches, R.n_patch, kSuperPatches,
                           R.n_super, R.supers);
        R.hypers = ws.get<Patch>("hypers", R.n_hyper);
        hipLaunchKernelGGL(k_sphere_of_spheres, dim3(R.n_hyper), dim3(64), 0, st, R.supers, R.n_super, kHyperSupers,
                           R.n_hyper, R.hypers);
        GBS_HIP(hipGetLastError());
    }

    // Device views of one pass of the table (copied in if the table is on the host).
    struct PassView {
        int64_t n_rays, n_segs;
        const int64_t* ray_ptr;   // absolute offsets
        const double* ray_w;
        const double *a, *t, *s0, *lo, *hi;
        const int64_t* face_ptr;  // absolute offsets into the full face_ids
        int64_t face_base;
        const int32_t* face_ids;  // starts at face_base
        const double* e1;         // frame vectors (anisotropic beams), or null
    };

    template <typename T>
    const T* stage(const std::string& name, const T* src, int64_t count, hipStream_t cs) {
        T* d = ws.get<T>(name, std::max<int64_t>(count, 1));
        if (count > 0) GBS_HIP(hipMemcpyAsync(d, src, sizeof(T) * count, hipMemcpyHostToDevice, cs));
        return d;
    }

    // Device view of one pass.  Host tables are copied into staging slot
    // `slot` on stream cs (the compute stream unless passes are overlapped).
    PassView view(const PassRange& ps, int slot = 0, hipStream_t cs = nullptr) {
        if (!cs) cs = st;
        const std::string sfx = std::to_string(slot);
        PassView v;
        v.n_rays = ps.ray_end - ps.ray_begin;
        v.n_segs = ps.seg_end - ps.seg_begin;
        const gbs_segs& S = *a.segs;
        if (!table_host()) {
            v.ray_ptr = a.rays->ray_ptr + ps.ray_begin;
            v.ray_w = a.rays->ray_w + ps.ray_begin;
            v.a = S.a + 3 * ps.seg_begin;
            v.t = S.t + 3 * ps.seg_begin;
            v.s0 = S.s0 + ps.seg_begin;
            v.lo = S.lo + ps.seg_begin;
            v.hi = S.hi + ps.seg_begin;
            v.face_ptr = S.face_ptr + ps.seg_begin;
            v.face_base = 0;
            v.face_ids = S.face_ids;
            v.e1 = S.e1 ? S.e1 + 3 * ps.seg_begin : nullptr;
            return v;
        }
        v.ray_ptr = stage("p_ray_ptr" + sfx, a.rays->ray_ptr + ps.ray_begin, v.n_rays + 1, cs);
        v.ray_w = stage("p_ray_w" + sfx, a.rays->ray_w + ps.ray_begin, v.n_rays, cs);
        v.a = stage("p_a" + sfx, S.a + 3 * ps.seg_begin, 3 * v.n_segs, cs);
        v.t = stage("p_t" + sfx, S.t + 3 * ps.seg_begin, 3 * v.n_segs, cs);
        v.s0 = stage("p_s0" + sfx, S.s0 + ps.seg_begin, v.n_segs, cs);
        v.lo = stage("p_lo" + sfx, S.lo + ps.seg_begin, v.n_segs, cs);
        v.hi = stage("p_hi" + sfx, S.hi + ps.seg_begin, v.n_segs, cs);
        v.face_ptr = stage("p_face_ptr" + sfx, S.face_ptr + ps.seg_begin, v.n_segs + 1, cs);
        v.face_base = ps.face_begin;
        v.face_ids = stage("p_face_ids" + sfx, S.face_ids ? S.face_ids + ps.face_begin : nullptr,
                           ps.face_end - ps.face_begin, cs);
        v.e1 = S.e1 && aniso() ? stage("p_e1" + sfx, S.e1 + 3 * ps.seg_begin, 3 * v.n_segs, cs) : nullptr;
        return v;
    }

    struct Lists {
        int32_t n_items = 0;
        const int64_t* src_cnt = nullptr;   // per source: first counter, pieces (item_cnt in the kernels)
        int64_t total = 0;
        const JobConst* jobs = nullptr;
        const SegRec* rec = nullptr;       // records in spatial order (what the kernels read)
        const FrameRec* frames = nullptr;  // anisotropic beams: ray frames in the same order
        SegRec* rec_raw = nullptr;         // records in table order (k_records writes them)
        const int32_t* seg_perm = nullptr; // spatial position -> table position
        const int32_t* seg_ray = nullptr;
        const int64_t* item_off = nullptr;
        const int32_t* item_order = nullptr;
        const int32_t* lists = nullptr;
        // pair-kernel work units (chunks of the item lists) and their partials
        const Work* work = nullptr;
        const int32_t* n_work = nullptr;     // device: number of work units
        const int32_t* item_wbase = nullptr;
        const int32_t* item_wcount = nullptr;
        double* partial = nullptr;
        int64_t work_cap = 0;
    };

    // Absolute end of the face ids a pass may read: the staged slice of a host
    // table; face_ptr[n_segs] on the device otherwise (none without face_ids).
    const int64_t* face_end_dev() const {
        return table_host() || !a.segs->face_ids ? nullptr : a.segs->face_ptr + a.segs->n_segs;
    }
    int64_t face_end_host(const PassRange& ps) const { return table_host() ? ps.face_end : 0; }

    // A pass planned up to its list total (plan_pass) and waiting to be
    // finished (finish_pass: lists, longest-first order, work units).
    struct Planned {
        Lists L;
        int slot = 0, cps = 0;
        int64_t n_cnt = 0, max_pieces = 0;
        const CullSplit* d_split = nullptr;
        const int32_t* d_nsplit = nullptr;
        const unsigned long long* hmask = nullptr;
        int64_t* off = nullptr;
        unsigned char* bat = nullptr;      // the count pass's batch records, replayed by the fill pass
        int64_t cap_r = 0;                 // records per region (whole blocks)
        const unsigned* bat_ctr = nullptr; // records handed out per region
        int32_t* heads = nullptr;
    };

    // Records per region of the cull's batch records (up to 8 bands): 1/8
    // above the most a region of this context has needed, 64 MiB in all
    // before any pass has run, at most GBS_CULL_RECORD_BYTES in all (default
    // 8 GiB; 0 turns the records off); none for the allocation-free forward.
    // The waves that do not fit are recomputed by the fill pass.
    int64_t cull_region_cap(int nb) const {
        if (ws.arena || nb == 0) return 0;
        const size_t stride = cull_batch_bytes(nb), regions = (size_t)cull_batch_regions();
        size_t limit = size_t(8) << 30;
        if (const char* e = std::getenv("GBS_CULL_RECORD_BYTES")) limit = (size_t)std::strtoull(e, nullptr, 10);
        const int64_t need = ctx->cull_region_need;
        const size_t want = need > 0 ? (size_t)(need + need / 8 + 2 * cull_batch_block()) * stride * regions
                                     : size_t(64) << 20;
        // whole blocks; block indices are int32
        const int64_t cap = std::min<int64_t>((int64_t)(std::min(want, limit) / (stride * regions)),
                                              INT32_MAX / (int64_t)regions);
        return cap / cull_batch_block() * cull_batch_block();
    }

    // Names of a pass's planning buffers: graph creation keeps every pass's
    // under its tag; a call's passes alternate between two slots, so that
    // the plan of pass i + 1 can be enqueued before pass i is finished.
    std::string slot_name(const char* base, int slot) const {
        return std::string(base) + (tag.empty() ? "%" + std::to_string(slot) : tag);
    }

    // Records, job constants, spatial order, the cull's count pass and the
    // scan of the counts for one pass; the list total and the status word
    // are copied to the slot's pinned words behind the slot's event.  No
    // synchronisation.
    Planned plan_pass(const PassRange& ps, const PassView& v, int pass_idx, unsigned long long* bmax = nullptr) {
        Planned P;
        P.slot = pass_idx % 2;
        Lists& L = P.L;
        const int64_t nseg = v.n_segs;
        int32_t* seg_ray = ws.get<int32_t>(slot_name("seg_ray", P.slot), nseg);
        SegRec* rec = ws.get<SegRec>(slot_name("rec", P.slot), nseg);
        if (nseg > 0) {
            hipLaunchKernelGGL(k_seg2ray, dim3(blocks_for(v.n_rays, 256)), dim3(256), 0, st, v.ray_ptr, v.n_rays,
                               ps.seg_begin, nseg, seg_ray);
            hipLaunchKernelGGL(k_records, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg, v.a, v.t, v.s0, v.lo,
                               v.hi, v.face_ptr, v.face_base, v.face_ids, a.faces->n_faces, a.faces->gamma, v.ray_w,
                               seg_ray, v.n_rays, face_end_dev(), face_end_host(ps), rec, status, bmax);
            GBS_HIP(hipGetLastError());
        }
        L.rec = rec;
        L.rec_raw = rec;
        L.seg_ray = seg_ray;
        JobConst* dJ = ws.get<JobConst>(slot_name("jobs", P.slot), n_jobs);
        if (n_jobs > 0) {
            hipLaunchKernelGGL(k_job_consts, dim3(blocks_for(n_jobs, 64)), dim3(64), 0, st, a.freqs, a.eps,
                               a.params->alpha, a.params->eps_e2, a.rays->n_src, a.n_freq, a.params->c,
                               a.params->gate_G, d_src_off, ps.seg_begin, ps.seg_end, dJ, status);
            GBS_HIP(hipGetLastError());
        }
        L.jobs = dJ;
        if (nseg > 0 && R.bbox) {
            // spatial order of the segments (each source's range stays in place)
            unsigned long long* k1 = ws.get<unsigned long long>("skeys", nseg);
            unsigned long long* k2 = ws.get<unsigned long long>("skeys2", nseg);
            int32_t* ids = ws.get<int32_t>("sids", nseg);
            int32_t* perm = ws.get<int32_t>(slot_name("seg_perm", P.slot), nseg);
            hipLaunchKernelGGL(k_seg_keys, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg, rec, dJ,
                               a.rays->n_src, a.n_freq, R.bbox, k1, ids);
            int end_bit = 32;
            while (end_bit < 64 && (1ll << (end_bit - 32)) < a.rays->n_src) ++end_bit;
            size_t tmp = 0;
            GBS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, k1, k2, ids, perm, (int)nseg, 0, end_bit, st));
            void* t = ws.get<char>("cub_tmp_segsort", tmp);
            GBS_HIP(hipcub::DeviceRadixSort::SortPairs(t, tmp, k1, k2, ids, perm, (int)nseg, 0, end_bit, st));
            SegRec* rs = ws.get<SegRec>(slot_name("rec_sorted", P.slot), nseg);
            hipLaunchKernelGGL(k_permute_rec, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg, rec, perm, rs);
            GBS_HIP(hipGetLastError());
            L.rec = rs;
            L.seg_perm = perm;
            rec = rs;
        }
        if (nseg > 0 && aniso()) {
            // ray frames (job independent): table order, then the records' order
            FrameRec* fr = ws.get<FrameRec>(slot_name("frames_raw", P.slot), nseg);
            hipLaunchKernelGGL(k_frames, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg, v.a, v.t, v.s0, v.e1,
                               fr, status);
            L.frames = fr;
            if (L.seg_perm) {
                FrameRec* fs = ws.get<FrameRec>(slot_name("frames", P.slot), nseg);
                hipLaunchKernelGGL(k_permute_frames, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg, fr,
                                   L.seg_perm, fs);
                L.frames = fs;
            }
            GBS_HIP(hipGetLastError());
        }
        const int64_t n_items = (int64_t)n_jobs * R.n_patch;
        GBS_CHECK(n_items < INT32_MAX, "too many work items");
        L.n_items = (int32_t)n_items;
        if (n_items == 0) return P;
        // split every source's segment range so that culling runs wide; one
        // workgroup culls one piece for all bands of its source.  The pieces
        // are laid out on the device (k_make_splits); the host sizes the grids
        // for the most pieces a pass can have: one cull wave per (super-patch,
        // piece), up to 256 pieces per source (more when there are fewer than
        // 128 super-patches) and about 64M list-length counters in all.  A piece holds 1,024 segments or more, down to 256
        // when a pass is too short for 32,768 cull waves (the waves near the
        // source set a short pass's time).  Each piece has one counter per
        // (band, patch) of its source; a source's counters are (band, patch,
        // piece) in that order from src_cnt[2 s], so the prefix sum of all
        // counters lays every (source, band, patch) list out as its pieces in
        // segment order
        const int n_src = a.rays->n_src, n_freq = a.n_freq;
        const int64_t cells = (int64_t)n_freq * R.n_patch;
        // few super-patches (impulse responses: a few thousand receivers,
        // many bands) take up to 32,768 / n_super pieces per source, so that
        // the cull still runs that many waves
        const int64_t per_src = std::max<int64_t>(256, 32768 / std::max<int64_t>(1, R.n_super));
        // a pass has at most n_src + budget pieces, fewer than 65,536
        const int64_t budget = std::max<int64_t>(
            1, std::min<int64_t>({per_src * n_src, ((int64_t(1) << 26) / cells) - n_src, 65535 - (int64_t)n_src}));
        int64_t span_min = 1024;
        while (span_min > kCullThreads && (int64_t)R.n_super * ((nseg + span_min - 1) / span_min) < 32768)
            span_min -= kCullThreads;
        int64_t span = std::max<int64_t>(span_min, (nseg + budget - 1) / budget);
        span = (span + kCullThreads - 1) / kCullThreads * kCullThreads;
        const int64_t n_span = std::max<int64_t>(1, (nseg + span - 1) / span);   // pieces per source, at most
        const int64_t max_pieces = std::min<int64_t>((int64_t)n_src * n_span, n_src + n_span);
        GBS_CHECK(max_pieces < 65536, "too many cull pieces");
        const int64_t n_cnt = cells * max_pieces;
        GBS_CHECK(n_cnt < INT32_MAX, "too many cull partitions");
        int32_t* counts = ws.get<int32_t>(slot_name("counts", P.slot), n_cnt + 2);
        int64_t* off = ws.get<int64_t>(slot_name("item_off", P.slot), n_cnt + 1);
        fill(st, (double*)counts, (n_cnt + 2) / 2, 0.0);
        CullSplit* d_split = ws.get<CullSplit>(slot_name("splits", P.slot), std::max<int64_t>(max_pieces, 1));
        int32_t* d_nsplit = ws.get<int32_t>(slot_name("n_splits", P.slot), 1);
        int64_t* src_cnt = ws.get<int64_t>(slot_name("src_cnt", P.slot), 2 * (size_t)n_src);
        hipLaunchKernelGGL(k_make_splits, dim3(1), dim3(64), 0, st, d_src_off, n_src, ps.seg_begin, ps.seg_end, span,
                           (int32_t)max_pieces, cells, d_split, d_nsplit, src_cnt);
        L.src_cnt = src_cnt;
        dim3 cg(R.n_super, (unsigned)std::max<int64_t>(max_pieces, 1));
        // batch records, shared by the passes of a slot (filled before the slot's next plan)
        const int nb = n_freq == 1 ? 1 : n_freq <= 4 ? 4 : n_freq <= 8 ? 8 : 0;
        P.cap_r = cull_region_cap(nb);
        const size_t n_ctr = (size_t)cull_batch_regions() * cull_batch_ctr_stride();
        P.bat = ws.get<unsigned char>("cull_batches%" + std::to_string(P.slot),
                                      P.cap_r > 0 ? (size_t)P.cap_r * cull_batch_regions() * cull_batch_bytes(nb) : 1);
        unsigned* bat_ctr = ws.get<unsigned>("cull_batch_ctr%" + std::to_string(P.slot), n_ctr + 2);
        P.bat_ctr = bat_ctr;
        P.heads = ws.get<int32_t>("cull_heads%" + std::to_string(P.slot), (size_t)2 * cg.x * cg.y);
        fill(st, (double*)bat_ctr, (n_ctr + 2) / 2, 0.0);
        // every chain starts empty (-1): the cull waves that level 0 leaves
        // without a segment end before they write theirs
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>(4096, blocks_for(2 * (int64_t)cg.x * cg.y, 256))),
                           dim3(256), 0, st, P.heads, 2 * (int64_t)cg.x * cg.y, (int32_t)-1);
        // up to 8 bands: band constants in wave-uniform registers, as many as needed
        auto cull_count = n_freq == 1 ? k_cull<false, 1> : n_freq <= 4 ? k_cull<false, 4>
                        : n_freq <= 8 ? k_cull<false, 8> : k_cull<false, 0>;
        auto cull_hyper = n_freq == 1 ? k_cull_hyper<1> : n_freq <= 4 ? k_cull_hyper<4>
                        : n_freq <= 8 ? k_cull_hyper<8> : k_cull_hyper<0>;
        // level 0: which segments of each chunk may reach each hyper-patch
        const int cps = (int)(span / kCullThreads);
        unsigned long long* hmask = ws.get<unsigned long long>(
            slot_name("hmask", P.slot), (size_t)std::max<int64_t>(max_pieces, 1) * cps * R.n_hyper * (kCullThreads / kWave));
        if (nseg > 0) {
            // level 0 also weighs each cull wave (piece, super-patch), or
            // each (piece, hyper-patch) where the super-patch tests would cost
            // too much (many segments and hyper-patches); the count pass starts
            // its waves heaviest first
            const int64_t n_waves = (int64_t)cg.x * cg.y, n_wt = n_waves;
            const int per_super = nseg * (int64_t)R.n_hyper <= (int64_t(1) << 24) ? 1 : 0;
            unsigned* weight = ws.get<unsigned>(slot_name("cull_weight", P.slot), n_wt + 32);
            int32_t* order = ws.get<int32_t>(slot_name("cull_order", P.slot), n_waves);
            hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)std::min<int64_t>(4096, blocks_for(n_wt + 32, 256))), dim3(256),
                               0, st, (int32_t*)weight, n_wt + 32, 0);
            hipLaunchKernelGGL(cull_hyper, dim3(cps, (unsigned)max_pieces), dim3(kCullThreads), 0, st, dJ, rec,
                               R.hypers, R.n_hyper, n_freq, cps, d_split, d_nsplit, hmask, R.supers, (int)R.n_super,
                               per_super, weight);
            hipLaunchKernelGGL(k_cull_order<false>, dim3(blocks_for(n_waves, 256)), dim3(256), 0, st, weight,
                               per_super, (int)R.n_super, (int)R.n_hyper, n_waves, weight + n_wt, order);
            hipLaunchKernelGGL(k_cull_order<true>, dim3(blocks_for(n_waves, 256)), dim3(256), 0, st, weight,
                               per_super, (int)R.n_super, (int)R.n_hyper, n_waves, weight + n_wt, order);
            hipLaunchKernelGGL(cull_count, cg, dim3(kWave), 0, st, dJ, rec, R.patches, R.supers, R.n_patch,
                               n_freq, src_cnt, d_split, d_nsplit, hmask, R.n_hyper, cps, counts, nullptr, nullptr,
                               P.bat, bat_ctr, P.cap_r, P.heads, order);
        }
        GBS_HIP(hipGetLastError());
        // counts are int32; accumulate in int64 through a converting iterator
        auto in64 = hipcub::TransformInputIterator<int64_t, Widen, const int32_t*>(counts, Widen());
        size_t tmp = 0;
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, in64, off, (int)(n_cnt + 1), st));
        void* t = ws.get<char>("cub_tmp_scan", tmp);
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(t, tmp, in64, off, (int)(n_cnt + 1), st));
        int64_t* words = ctx->plan_words + 3 * P.slot;
        words[1] = 0;
        words[2] = 0;
        GBS_HIP(hipMemcpyAsync(words, off + n_cnt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipMemcpyAsync(words + 1, status, sizeof(int), hipMemcpyDeviceToHost, st));
        hipLaunchKernelGGL(k_cull_need, dim3(1), dim3(cull_batch_regions()), 0, st, bat_ctr, bat_ctr + n_ctr);
        GBS_HIP(hipMemcpyAsync(words + 2, bat_ctr + n_ctr, sizeof(unsigned), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipEventRecord(ctx->planned[P.slot], st));
        P.n_cnt = n_cnt;
        P.max_pieces = max_pieces;
        P.cps = cps;
        P.d_split = d_split;
        P.d_nsplit = d_nsplit;
        P.hmask = hmask;
        P.off = off;
        return P;
    }

    // Waits for a planned pass's list total (the host's one synchronisation
    // per pass, on work enqueued before it), checks the status word, then
    // fills the lists and lays out the work units.
    Lists finish_pass(const Planned& P) {
        Lists L = P.L;
        if (L.n_items == 0) return L;
        GBS_HIP(hipEventSynchronize(ctx->planned[P.slot]));
        const int64_t* words = ctx->plan_words + 3 * P.slot;
        L.total = words[0];
        ctx->cull_region_need = std::max(ctx->cull_region_need, words[2]);
        check_status((int)words[1]);     // before any list is filled or any pair kernel runs
        const int n_freq = a.n_freq;
        const int64_t n_items = L.n_items;
        const SegRec* rec = L.rec;
        int32_t* lists = ws.get<int32_t>(slot_name("lists", P.slot), std::max<int64_t>(L.total, 1));
        auto cull_fill = n_freq == 1 ? k_cull<true, 1> : n_freq <= 4 ? k_cull<true, 4>
                       : n_freq <= 8 ? k_cull<true, 8> : k_cull<true, 0>;
        dim3 cg(R.n_super, (unsigned)std::max<int64_t>(P.max_pieces, 1));
        if (L.total > 0) {
            // recorded waves are replayed; k_cull recomputes the others, and
            // runs only when a region ran out of records (or none were kept)
            auto replay = n_freq == 1 ? k_cull_replay<1> : n_freq <= 4 ? k_cull_replay<4>
                        : n_freq <= 8 ? k_cull_replay<8> : nullptr;
            // one wave per block: as many blocks as the fullest region handed out
            const int64_t n_blk = (std::min<int64_t>(words[2], P.cap_r) + cull_batch_block() - 1) / cull_batch_block();
            if (replay && P.cap_r > 0 && n_blk > 0)
                hipLaunchKernelGGL(replay, dim3((unsigned)n_blk, (unsigned)cull_batch_regions()), dim3(kWave), 0, st,
                                   P.d_split, (int)R.n_super, R.n_patch, n_freq, L.src_cnt, P.off, P.bat, P.bat_ctr,
                                   P.cap_r, P.heads, lists);
            if (!replay || words[2] > P.cap_r)
                hipLaunchKernelGGL(cull_fill, cg, dim3(kWave), 0, st, L.jobs, rec, R.patches, R.supers, R.n_patch,
                                   n_freq, L.src_cnt, P.d_split, P.d_nsplit, P.hmask, R.n_hyper, P.cps, nullptr, P.off,
                                   lists, P.bat, nullptr, P.cap_r, P.heads, nullptr);
        }
        GBS_HIP(hipGetLastError());
        int64_t* off = P.off;
        // longest lists first, unless the units are short enough that their
        // order cannot leave a long one for the end (items keep their order)
        const int chunk = work_chunk();
        int32_t* lens = ws.get<int32_t>("lens", n_items);
        hipLaunchKernelGGL(k_item_lengths, dim3(blocks_for(n_items, 256)), dim3(256), 0, st, off, (int32_t)n_items,
                           R.n_patch, n_freq, L.src_cnt, lens);
        int32_t* ids = ws.get<int32_t>("oids", n_items);
        int32_t* order = ids;
        hipLaunchKernelGGL(k_iota, dim3(blocks_for(n_items, 256)), dim3(256), 0, st, ids, (int32_t)n_items);
        if (chunk > kWorkChunkPasses) {
            int32_t* keys2 = ws.get<int32_t>("okeys", n_items);
            order = ws.get<int32_t>("order", n_items);
            size_t tmp2 = 0;
            GBS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp2, lens, keys2, ids, order,
                                                                 (int)n_items, 0, 32, st));
            void* t2 = ws.get<char>("cub_tmp_order", tmp2);
            GBS_HIP(hipcub::DeviceRadixSort::SortPairsDescending(t2, tmp2, lens, keys2, ids, order, (int)n_items, 0,
                                                                 32, st));
        }
        // work units: every list cut into chunks of at most `chunk` segments
        const int64_t cap = n_items + L.total / chunk + 1;
        GBS_CHECK(cap < INT32_MAX, "too many work units");
        int32_t* nw = ws.get<int32_t>("nwork", n_items + 1);
        int32_t* wb = ws.get<int32_t>("wbase", n_items + 1);
        hipLaunchKernelGGL(k_work_counts, dim3(blocks_for(n_items + 1, 256)), dim3(256), 0, st, order, lens,
                           (int32_t)n_items, chunk, nw);
        size_t tmp3 = 0;
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp3, nw, wb, (int)(n_items + 1), st));
        void* t3 = ws.get<char>("cub_tmp_work", tmp3);
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(t3, tmp3, nw, wb, (int)(n_items + 1), st));
        Work* work = ws.get<Work>(slot_name("work", P.slot), cap);
        int32_t* iwb = ws.get<int32_t>(slot_name("item_wbase", P.slot), n_items);
        int32_t* iwc = ws.get<int32_t>(slot_name("item_wcount", P.slot), n_items);
        int32_t* n_work = ws.get<int32_t>(slot_name("n_work", P.slot), 1);
        hipLaunchKernelGGL(k_make_work, dim3(blocks_for(n_items, 256)), dim3(256), 0, st, order, off, R.n_patch,
                           n_freq, L.src_cnt, wb,
                           (int32_t)n_items, chunk, work, iwb, iwc, n_work);
        GBS_HIP(hipGetLastError());
        L.work = work;
        L.n_work = n_work;
        L.item_wbase = iwb;
        L.item_wcount = iwc;
        L.work_cap = cap;
        L.item_off = off;
        L.item_order = order;
        L.lists = lists;
        return L;
    }

    // Plans and finishes one pass (one synchronisation).
    Lists build_lists(const PassRange& ps, const PassView& v, int pass_idx, unsigned long long* bmax = nullptr) {
        return finish_pass(plan_pass(ps, v, pass_idx, bmax));
    }

    struct Widen {
        __host__ __device__ int64_t operator()(const int32_t& x) const { return (int64_t)x; }
    };
};

// HIP events around a stretch of work on the context stream (only when
// timing was requested; end() synchronises on the stop event).
struct EventPair {
    bool on;
    hipEvent_t a = nullptr, b = nullptr;
    explicit EventPair(bool enabled) : on(enabled) {
        if (on) {
            GBS_HIP(hipEventCreate(&a));
            GBS_HIP(hipEventCreate(&b));
        }
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    bool stopped = false;
    void begin(hipStream_t st) {
        if (on) GBS_HIP(hipEventRecord(a, st));
        stopped = false;
    }
    // Records the stop event now; end() then only waits for it.
    void stop(hipStream_t st) {
        if (on) GBS_HIP(hipEventRecord(b, st));
        stopped = true;
    }
    double end(hipStream_t st) {
        if (!on) return 0.0;
        if (!stopped) GBS_HIP(hipEventRecord(b, st));
        stopped = false;
        GBS_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        GBS_HIP(hipEventElapsedTime(&ms, a, b));
        return ms;
    }
};

int pick_nr(gbs_ctx* ctx, const gbs_params* p, int64_t n_rcv) {
    if (p->rcv_per_lane) return p->rcv_per_lane;
    if (ctx->tuned_nr[p->mode]) return ctx->tuned_nr[p->mode];
    (void)n_rcv;
    return 1;   // measured fastest on MI355X: 64-receiver patches cull tightest
}

// Workgroups of the persistent kernels: as many as can be resident at once
// (every wave of a workgroup pops its own items), never more than needed.
int64_t persistent_grid(gbs_ctx* ctx, const void* kern, int64_t n_items) {
    int per_cu = 0;
    GBS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kPairThreads, 0));
    int64_t grid = std::max(1, per_cu) * (int64_t)ctx->n_cu;
    const int64_t waves = kPairThreads / kWave;
    grid = std::min<int64_t>(grid, (n_items + waves - 1) / waves);
    ctx->stats.grid = (int32_t)grid;
    ctx->stats.blocks_per_cu = per_cu;
    return std::max<int64_t>(grid, 1);
}

// Adds a pass's partial sums into P in work-unit order (write: the call's
// only pass, which writes P and TL instead).
void reduce_pass(hipStream_t st, const Planner::Lists& L, const RcvPlan& R, int nr, int64_t n_rcv, double* P,
                 double* TL, bool write) {
    const int64_t threads = (int64_t)L.n_items * 64 * nr;
    hipLaunchKernelGGL(k_reduce_partials, dim3(blocks_for(threads, 256)), dim3(256), 0, st, L.jobs, L.item_wbase,
                       L.item_wcount, L.n_items, R.n_patch, nr, R.perm, n_rcv, L.partial, P, TL, (int)write);
    GBS_HIP(hipGetLastError());
}

template <int MODE, int NR, bool COUNT>
void launch_pairs(gbs_ctx* ctx, hipStream_t st, const Planner::Lists& L, const RcvPlan& R, int64_t n_rcv, double* P,
                  unsigned* ctr, unsigned long long* n_active, EventPair* ev, double* TL, bool write, bool reduce) {
    auto kern = k_pairs<MODE, NR, COUNT>;
    const int64_t grid = persistent_grid(ctx, (const void*)kern, L.work_cap);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, ctr);
    if (ev) ev->begin(st);
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPairThreads), 0, st, L.jobs, L.work, L.n_work, R.n_patch, ctr,
                       L.lists, L.rec, L.frames, R.rx, R.ry, R.rz, R.r2, L.partial, n_active);
    GBS_HIP(hipGetLastError());
    if (ev) ev->stop(st);
    if (reduce) reduce_pass(st, L, R, NR, n_rcv, P, TL, write);
}

template <int MODE, bool COUNT>
void dispatch_nr(int nr, gbs_ctx* ctx, hipStream_t st, const Planner::Lists& L, const RcvPlan& R, int64_t n_rcv,
                 double* P, unsigned* ctr, unsigned long long* na, EventPair* ev, double* TL, bool write,
                 bool reduce) {
    if (nr == 1) launch_pairs<MODE, 1, COUNT>(ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce);
    else if (nr == 2) launch_pairs<MODE, 2, COUNT>(ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce);
    else launch_pairs<MODE, 4, COUNT>(ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce);
}

template <int MODE>
void dispatch_count(bool count, int nr, gbs_ctx* ctx, hipStream_t st, const Planner::Lists& L, const RcvPlan& R,
                    int64_t n_rcv, double* P, unsigned* ctr, unsigned long long* na, EventPair* ev, double* TL,
                    bool write, bool reduce) {
    count ? dispatch_nr<MODE, true>(nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce)
          : dispatch_nr<MODE, false>(nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce);
}

// mode: GBS_MODE_*; absorb: some job has atmospheric absorption (the kernel
// variant with the absorption exponent; the others skip it); aniso:
// anisotropic beams (counting counts the exact gate's pairs).
// ev (optional): HIP events around the pair kernel's launch alone.
// write: the call's only pass; the reduction writes every output of P (no
// zero fill before it) and, with TL, the transmission loss.  reduce: false
// leaves the partial sums for reduce_pass on another stream.
void dispatch_pairs(int mode, bool absorb, bool aniso, bool count, int nr, gbs_ctx* ctx, hipStream_t st,
                    const Planner::Lists& L, const RcvPlan& R, int64_t n_rcv, double* P, unsigned* ctr,
                    unsigned long long* na, EventPair* ev = nullptr, double* TL = nullptr, bool write = false,
                    bool reduce = true) {
    GBS_CHECK(L.partial != nullptr, "work-unit partials not allocated");
    const int m = (mode == GBS_MODE_F64 ? 0 : mode == GBS_MODE_MIX ? 1 : 2) | (absorb ? 4 : 0);
    if (aniso) {
        switch (m) {
            case 0: dispatch_count<8>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
            case 1: dispatch_count<9>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
            case 2: dispatch_count<10>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
            case 4: dispatch_count<12>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
            case 5: dispatch_count<13>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
            default: dispatch_count<14>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        }
        return;
    }
    switch (m) {
        case 0: dispatch_count<0>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        case 1: dispatch_count<1>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        case 2: dispatch_count<2>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        case 4: dispatch_count<4>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        case 5: dispatch_count<5>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
        default: dispatch_count<6>(count, nr, ctx, st, L, R, n_rcv, P, ctr, na, ev, TL, write, reduce); break;
    }
}


// The copy stream and its events, created on first use (default priority).
void ensure_copy_stream(gbs_ctx* ctx) {
    if (ctx->copy_stream) return;
    GBS_HIP(hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        GBS_HIP(hipEventCreateWithFlags(&ctx->copied[i], hipEventDisableTiming));
        GBS_HIP(hipEventCreateWithFlags(&ctx->released[i], hipEventDisableTiming));
    }
    ctx->ws->copy_stream = ctx->copy_stream;
}

// The pair streams and their events, created on first use (default priority).
void ensure_pair_streams(gbs_ctx* ctx, Workspace& ws) {
    for (int i = 0; i < 2; ++i) {
        if (!ctx->pair_stream[i]) {
            GBS_HIP(hipStreamCreateWithFlags(&ctx->pair_stream[i], hipStreamNonBlocking));
            GBS_HIP(hipEventCreateWithFlags(&ctx->pair_ready[i], hipEventDisableTiming));
            GBS_HIP(hipEventCreateWithFlags(&ctx->pair_done[i], hipEventDisableTiming));
        }
        ws.pair_streams[i] = ctx->pair_stream[i];
    }
}

int forward_impl(gbs_ctx* ctx, Workspace& ws, const Args& a, double* P, double* TL, int nr_override,
                 int chunk_override = 0) {
    validate_host(a);
    GBS_CHECK(P || (int64_t)a.rays->n_src * a.n_freq * a.n_rcv == 0, "null P");
    const int nr = nr_override ? nr_override : pick_nr(ctx, a.params, a.n_rcv);
    Planner pl(ctx, ws, a, nr);
    pl.chunk_override = chunk_override;
    hipStream_t st = ctx->stream;
    const int64_t n_out = (int64_t)pl.n_jobs * a.n_rcv;
    // P is zeroed before a call in several passes accumulates into it; a
    // call's only pass writes all of it (and TL) in its reduction
    bool zeroed = false, tl_done = false;
    auto zero_P = [&]() {
        if (!zeroed) fill(st, P, 2 * n_out, 0.0);
        zeroed = true;
    };
    gbs_stats stats{};
    stats.patch_rcv = 64 * nr;
    if (n_out > 0 && a.segs->n_segs > 0) {
        pl.reset_status();
        // the receivers' planning first: the device works on it while the
        // host checks a host table and lays out its passes
        pl.plan_receivers(64 * nr);
        pl.source_offsets();
        stats.dense_pairs = a.segs->n_segs * a.n_rcv * a.n_freq;   // every segment belongs to one source
        pl.make_passes();
        unsigned* ctr = ws.get<unsigned>("ctr", 1);
        const bool count = (a.params->flags & GBS_FLAG_COUNT_ACTIVE) != 0;
        unsigned long long* na = ws.get<unsigned long long>("n_active", 1);
        if (count) GBS_HIP(hipMemsetAsync(na, 0, sizeof(unsigned long long), st));
        const bool timed = (a.params->flags & GBS_FLAG_TIME_KERNELS) != 0;
        EventPair ev_pairs(timed), ev_cull(timed);
        // Several passes: pass i + 1 is planned (up to its list total) before
        // pass i's lists are filled, so the host's wait for pass i's total
        // covers only work that was enqueued before it, and the host enqueues
        // pass i's lists and pair kernel while the device still plans; a
        // timed call plans pass by pass.  Host tables: pass i + 2 is copied on
        // the copy stream into the staging slot of pass i as soon as pass i's
        // records are built (the pair kernel never reads the staged table).
        const size_t n_pass = pl.passes.size();
        const bool one_pass = n_pass == 1;
        if (!one_pass) zero_P();
        const bool overlap = pl.table_host() && n_pass > 1;
        const bool pipe = n_pass > 1 && !timed;
        Planner::PassView views[2];
        auto issue = [&](size_t pi) {
            const int slot = (int)(pi % 2);
            if (pi >= 2) GBS_HIP(hipStreamWaitEvent(ctx->copy_stream, ctx->released[slot], 0));
            views[slot] = pl.view(pl.passes[pi], slot, ctx->copy_stream);
            GBS_HIP(hipEventRecord(ctx->copied[slot], ctx->copy_stream));
        };
        Planner::Planned pend[2];
        auto start = [&](size_t pi) {
            Planner::PassView v;
            if (overlap) {
                GBS_HIP(hipStreamWaitEvent(st, ctx->copied[pi % 2], 0));
                v = views[pi % 2];
            } else {
                v = pl.view(pl.passes[pi]);
            }
            pend[pi % 2] = pl.plan_pass(pl.passes[pi], v, (int)pi);
            if (overlap) {
                GBS_HIP(hipEventRecord(ctx->released[pi % 2], st));
                if (pi + 2 < n_pass) issue(pi + 2);
            }
        };
        if (overlap) {
            ensure_copy_stream(ctx);
            issue(0);
            issue(1);
        }
        if (pipe) {
            start(0);
            start(1);
        }
        // Several passes, untimed and uncounted: pass i's pair kernel runs on
        // pair_stream[i % 2] once its lists are laid out, and pass i + 1's
        // lists are laid out meanwhile, so that its pair kernel fills the
        // GPU as pass i's drains; the partial sums are added into P on the
        // compute stream, pass by pass, and a slot is planned again only
        // after its pair kernel and reduction
        const bool spread = pipe && !count;
        if (spread) {
            ensure_pair_streams(ctx, ws);
            Planner::Lists Ls[2];
            bool has[2] = {false, false};
            auto finish_and_launch = [&](size_t pi) {
                const int slot = (int)(pi % 2);
                Planner::Lists L = pl.finish_pass(pend[slot]);
                stats.listed_pairs += L.total * (int64_t)pl.R.per;
                stats.n_items += L.n_items;
                has[slot] = L.n_items > 0 && L.total > 0;
                if (has[slot]) {
                    L.partial = ws.get<double>(pl.slot_name("partial", slot), L.work_cap * nr * 64 * 2);
                    unsigned* c = ws.get<unsigned>(pl.slot_name("ctr", slot), 1);
                    hipStream_t ps = ctx->pair_stream[slot];
                    GBS_HIP(hipEventRecord(ctx->pair_ready[slot], st));
                    GBS_HIP(hipStreamWaitEvent(ps, ctx->pair_ready[slot], 0));
                    dispatch_pairs(a.params->mode, pl.absorb(), pl.aniso(), false, nr, ctx, ps, L, pl.R, a.n_rcv, P,
                                   c, na, nullptr, nullptr, false, false);
                    GBS_HIP(hipEventRecord(ctx->pair_done[slot], ps));
                }
                Ls[slot] = L;
            };
            finish_and_launch(0);
            for (size_t pi = 0; pi < n_pass; ++pi) {
                const int slot = (int)(pi % 2);
                if (pi + 1 < n_pass) finish_and_launch(pi + 1);
                if (has[slot]) {
                    GBS_HIP(hipStreamWaitEvent(st, ctx->pair_done[slot], 0));
                    reduce_pass(st, Ls[slot], pl.R, nr, a.n_rcv, P, nullptr, false);
                }
                if (pi + 2 < n_pass) start(pi + 2);
            }
        }
        for (size_t pi = 0; pi < (spread ? 0 : n_pass); ++pi) {
            ev_cull.begin(st);
            if (!pipe) start(pi);
            Planner::Lists L = pl.finish_pass(pend[pi % 2]);
            stats.ms_cull += ev_cull.end(st);
            stats.listed_pairs += L.total * (int64_t)pl.R.per;
            stats.n_items += L.n_items;
            if (L.n_items > 0 && L.total > 0) {
                L.partial = ws.get<double>("partial", L.work_cap * nr * 64 * 2);
                dispatch_pairs(a.params->mode, pl.absorb(), pl.aniso(), count, nr, ctx, st, L, pl.R, a.n_rcv, P, ctr, na,
                               timed ? &ev_pairs : nullptr, one_pass ? TL : nullptr, one_pass);
                if (one_pass) {
                    zeroed = true;
                    tl_done = TL != nullptr;
                }
                stats.ms_pairs += ev_pairs.end(st);
            }
            if (pipe && pi + 2 < n_pass) start(pi + 2);
        }
        stats.n_chunks = (int32_t)pl.passes.size();
        zero_P();                         // a call with nothing to reduce
        if (count) {
            unsigned long long h = 0;
            GBS_HIP(hipMemcpyAsync(&h, na, sizeof(h), hipMemcpyDeviceToHost, st));
            GBS_HIP(hipStreamSynchronize(st));
            stats.active_pairs = (int64_t)h;
        }
    } else {
        zero_P();
        pl.check_jobs_on_host();
    }
    if (TL && n_out > 0 && !tl_done) {
        hipLaunchKernelGGL(k_tl, dim3(blocks_for(n_out, 256)), dim3(256), 0, st, P, n_out, TL);
        GBS_HIP(hipGetLastError());
    }
    stats.grid = ctx->stats.grid;
    stats.blocks_per_cu = ctx->stats.blocks_per_cu;
    stats.scratch_bytes = (int64_t)ws.held();
    ctx->stats = stats;
    return GBS_OK;
}

// ------------------------------------------------------------ ray tracing
// Groups of kTraceGroup boxes in Morton order of their centres, each with the
// union of its members' bounds.
struct TraceScene {
    std::vector<double> gbox;         // [n_groups * 6]
    std::vector<int32_t> members;     // [n_groups * kTraceGroup], -1 = empty
    int n_groups = 0;
};

TraceScene group_boxes(const std::vector<double>& bx, int n_boxes) {
    TraceScene S;
    if (n_boxes == 0) return S;
    double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY};
    for (int b = 0; b < n_boxes; ++b)
        for (int j = 0; j < 2; ++j) {
            lo[j] = std::min(lo[j], bx[5 * b + 2 * j]);
            hi[j] = std::max(hi[j], bx[5 * b + 2 * j + 1]);
        }
    auto spread = [](uint32_t v) {                 // 16 bits -> every other bit
        v &= 0xffffu;
        v = (v | (v << 8)) & 0x00ff00ffu;
        v = (v | (v << 4)) & 0x0f0f0f0fu;
        v = (v | (v << 2)) & 0x33333333u;
        v = (v | (v << 1)) & 0x55555555u;
        return v;
    };
    std::vector<std::pair<uint32_t, int32_t>> key(n_boxes);
    for (int b = 0; b < n_boxes; ++b) {
        uint32_t q[2];
        for (int j = 0; j < 2; ++j) {
            const double c = 0.5 * (bx[5 * b + 2 * j] + bx[5 * b + 2 * j + 1]);
            const double w = hi[j] > lo[j] ? (c - lo[j]) / (hi[j] - lo[j]) : 0.0;
            q[j] = (uint32_t)std::min(65535.0, std::max(0.0, w * 65535.0));
        }
        key[b] = {spread(q[0]) | (spread(q[1]) << 1), b};
    }
    std::sort(key.begin(), key.end());
    S.n_groups = (n_boxes + kTraceGroup - 1) / kTraceGroup;
    S.gbox.assign((size_t)S.n_groups * 6, 0.0);
    S.members.assign((size_t)S.n_groups * kTraceGroup, -1);
    for (int g = 0; g < S.n_groups; ++g) {
        double glo[3] = {INFINITY, INFINITY, 0.0}, ghi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int m = 0; m < kTraceGroup && g * kTraceGroup + m < n_boxes; ++m) {
            const int b = key[g * kTraceGroup + m].second;
            S.members[g * kTraceGroup + m] = b;
            glo[0] = std::min(glo[0], bx[5 * b]);
            ghi[0] = std::max(ghi[0], bx[5 * b + 1]);
            glo[1] = std::min(glo[1], bx[5 * b + 2]);
            ghi[1] = std::max(ghi[1], bx[5 * b + 3]);
            ghi[2] = std::max(ghi[2], bx[5 * b + 4]);
        }
        for (int j = 0; j < 3; ++j) {
            S.gbox[6 * g + j] = glo[j];
            S.gbox[6 * g + 3 + j] = ghi[j];
        }
    }
    return S;
}

struct TraceOut {
    int64_t* ray_ptr;
    double *a, *t, *s0, *lo, *hi;
    int64_t* face_ptr;
    int32_t* face_ids;
    double* e1;          // optional: the carried ray frame (needs fan.e1)
};

// What a count token stands for: the arguments of the counted call.
std::vector<uint64_t> trace_signature(const gbs_scene* sc, const gbs_fan* fan) {
    auto ptr = [](const void* p) { return (uint64_t)(uintptr_t)p; };
    uint64_t smax_bits = 0;
    std::memcpy(&smax_bits, &sc->s_max, sizeof smax_bits);
    return {(uint64_t)sc->n_boxes, (uint64_t)sc->panels, ptr(sc->boxes), smax_bits, (uint64_t)sc->max_refl,
            (uint64_t)sc->image_complete, (uint64_t)fan->n_src, ptr(fan->src_xyz), (uint64_t)fan->n_rays,
            ptr(fan->dirs), ptr(fan->ray_src), ptr(fan->s_max_src), ptr(fan->e1)};
}

// Count pass and prefix sums; with `out` also the write pass (after the
// capacity check).  With a token from the last count of the same arguments,
// the count is reused.  Returns the sizes.
std::pair<int64_t, int64_t> trace_impl(gbs_ctx* ctx, const gbs_scene* sc, const gbs_fan* fan, int64_t cap_segs,
                                       int64_t cap_faces, const TraceOut* out, int64_t token = 0) {
    GBS_CHECK(sc && fan, "scene and fan must be non-null");
    const bool reuse = out && token != 0;
    if (reuse) {
        GBS_CHECK(token == ctx->trace_token, "count token is not the last gbs_trace_count on this context");
        GBS_CHECK(trace_signature(sc, fan) == ctx->trace_sig, "count token was issued for other arguments");
    }
    ctx->trace_token = 0;                 // the workspace is about to change
    GBS_CHECK(sc->n_boxes >= 0 && (sc->n_boxes == 0 || sc->boxes), "scene.boxes");
    GBS_CHECK(sc->panels >= 1 && sc->panels <= 8, "scene.panels must be in 1..8");
    GBS_CHECK(sc->max_refl >= 0 && sc->max_refl <= kTraceMaxRefl, "scene.max_refl must be in 0..32");
    GBS_CHECK(std::isfinite(sc->s_max) && sc->s_max > 0, "scene.s_max must be finite and > 0");
    GBS_CHECK(sc->image_complete == 0 || sc->image_complete == 1, "scene.image_complete must be 0 or 1");
    GBS_CHECK(!sc->image_complete || sc->n_boxes == 0, "image completion is defined for the open plane only");
    GBS_CHECK(fan->n_src >= 1 && fan->src_xyz, "fan.src_xyz");
    GBS_CHECK(fan->n_rays >= 0 && (fan->n_rays == 0 || fan->dirs), "fan.dirs");
    GBS_CHECK(fan->n_rays < INT32_MAX - 1, "fan.n_rays too large");
    const double faces_total = 1.0 + (double)sc->n_boxes * 5.0 * sc->panels * sc->panels;
    GBS_CHECK(faces_total < (double)INT32_MAX, "too many faces");
    hipStream_t st = ctx->stream;
    Workspace& ws = *ctx->ws;
    // small tables to the host: validation and box groups
    std::vector<double> bx((size_t)sc->n_boxes * 5), src((size_t)fan->n_src * 3);
    std::vector<double> smax(fan->s_max_src ? fan->n_src : 0);
    if (sc->n_boxes)
        GBS_HIP(hipMemcpyAsync(bx.data(), sc->boxes, bx.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    GBS_HIP(hipMemcpyAsync(src.data(), fan->src_xyz, src.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    if (fan->s_max_src)
        GBS_HIP(hipMemcpyAsync(smax.data(), fan->s_max_src, smax.size() * sizeof(double), hipMemcpyDeviceToHost,
                               st));
    GBS_HIP(hipStreamSynchronize(st));
    for (double v : smax) GBS_CHECK(std::isfinite(v) && v > 0, "fan.s_max_src must be finite and > 0");
    for (int b = 0; b < sc->n_boxes; ++b) {
        const double* q = &bx[5 * b];
        GBS_CHECK(std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]) && std::isfinite(q[3]) &&
                      std::isfinite(q[4]) && q[0] < q[1] && q[2] < q[3] && q[4] > 0,
                  "box " + std::to_string(b) + " must be finite with x0 < x1, y0 < y1, h > 0");
    }
    for (int k = 0; k < fan->n_src; ++k)
        GBS_CHECK(std::isfinite(src[3 * k]) && std::isfinite(src[3 * k + 1]) && std::isfinite(src[3 * k + 2]) &&
                      src[3 * k + 2] > 0,
                  "sources must be finite and above the ground");
    const int64_t n = fan->n_rays;
    const TraceScene S = reuse ? TraceScene{} : group_boxes(bx, sc->n_boxes);
    const int n_groups = reuse ? ctx->trace_groups : S.n_groups;
    const size_t ng = std::max<size_t>(n_groups, 1);
    double* d_box = ws.get<double>("tr_box", std::max<size_t>(bx.size(), 1));
    double* d_gbox = ws.get<double>("tr_gbox", ng * 6);
    int32_t* d_mem = ws.get<int32_t>("tr_members", ng * kTraceGroup);
    if (!reuse && !bx.empty())
        GBS_HIP(hipMemcpyAsync(d_box, bx.data(), bx.size() * sizeof(double), hipMemcpyHostToDevice, st));
    if (!reuse && S.n_groups) {
        GBS_HIP(hipMemcpyAsync(d_gbox, S.gbox.data(), S.gbox.size() * sizeof(double), hipMemcpyHostToDevice, st));
        GBS_HIP(hipMemcpyAsync(d_mem, S.members.data(), S.members.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               st));
    }
    int64_t* nseg = ws.get<int64_t>("tr_nseg", n + 1);
    int64_t* nface = ws.get<int64_t>("tr_nface", n + 1);
    int64_t* rp = out ? out->ray_ptr : ws.get<int64_t>("tr_rayptr", n + 1);
    int64_t* fbase = ws.get<int64_t>("tr_fbase", n + 1);
    const dim3 grid(blocks_for(n, kTraceThreads)), block(kTraceThreads);
    int64_t tot[2] = {0, 0};
    if (reuse) {
        // the offsets of the counted call, into the caller's ray_ptr
        GBS_HIP(hipMemcpyAsync(rp, ws.get<int64_t>("tr_rayptr", n + 1), sizeof(int64_t) * (n + 1),
                               hipMemcpyDeviceToDevice, st));
        tot[0] = ctx->trace_tot[0];
        tot[1] = ctx->trace_tot[1];
    } else {
        int* bad = ws.get<int>("tr_bad", 1);
        GBS_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
        GBS_HIP(hipMemsetAsync(nseg + n, 0, sizeof(int64_t), st));
        if (n > 0)
            hipLaunchKernelGGL(k_trace<true>, grid, block, 0, st, n, fan->n_src, fan->src_xyz, fan->ray_src, fan->dirs,
                               fan->s_max_src, d_box, d_gbox, d_mem, S.n_groups, sc->panels, sc->max_refl, sc->s_max,
                               sc->image_complete, nseg, bad,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                               fan->e1, nullptr);
        GBS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_trace_face_counts, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, n, nseg, nface);
        size_t tmp = 0;
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, nseg, rp, (int)(n + 1), st));
        void* tb = ws.get<char>("tr_scan", tmp);
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(tb, tmp, nseg, rp, (int)(n + 1), st));
        GBS_HIP(hipcub::DeviceScan::ExclusiveSum(tb, tmp, nface, fbase, (int)(n + 1), st));
        int h_bad = 0;
        GBS_HIP(hipMemcpyAsync(&tot[0], rp + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipMemcpyAsync(&tot[1], fbase + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipMemcpyAsync(&h_bad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipStreamSynchronize(st));
        GBS_CHECK(!(h_bad & 1), "fan.dirs must be unit vectors");
        GBS_CHECK(!(h_bad & 2), "fan.ray_src must be non-decreasing and in [0, n_src)");
        GBS_CHECK(!(h_bad & 4), "fan.e1 must be unit vectors normal to the directions");
        if (!out) {
            ctx->trace_token = ++ctx->trace_token_next;
            ctx->trace_sig = trace_signature(sc, fan);
            ctx->trace_tot[0] = tot[0];
            ctx->trace_tot[1] = tot[1];
            ctx->trace_groups = S.n_groups;
            return {tot[0], tot[1]};
        }
    }
    GBS_CHECK(tot[0] <= cap_segs && tot[1] <= cap_faces,
              "table capacity too small: needs " + std::to_string(tot[0]) + " segments and " +
                  std::to_string(tot[1]) + " face ids");
    GBS_CHECK(tot[0] == 0 || (out->a && out->t && out->s0 && out->lo && out->hi && out->face_ptr),
              "table outputs must be non-null");
    GBS_CHECK(tot[1] == 0 || out->face_ids, "face_ids must be non-null");
    GBS_CHECK(out->face_ptr, "face_ptr must be non-null");
    GBS_CHECK(!out->e1 || fan->e1, "the frame output needs launch frames (fan.e1)");
    if (n > 0)
        hipLaunchKernelGGL(k_trace<false>, grid, block, 0, st, n, fan->n_src, fan->src_xyz, fan->ray_src,
                           fan->dirs, fan->s_max_src, d_box, d_gbox, d_mem, n_groups, sc->panels, sc->max_refl,
                           sc->s_max, sc->image_complete,
                           nullptr, nullptr, rp, fbase, out->a, out->t, out->s0, out->lo, out->hi, out->face_ptr,
                           out->face_ids, fan->e1, out->e1);
    hipLaunchKernelGGL(k_trace_close, dim3(1), dim3(64), 0, st, fbase, n, tot[0], out->face_ptr);
    GBS_HIP(hipGetLastError());
    return {tot[0], tot[1]};
}

}  // namespace

// =================================================================== C ABI
extern "C" {

int gbs_version(void) { return GBS_VERSION; }

// ISO 9613-1 pure-tone attenuation: molar concentration of water vapour h
// from the saturation pressure over the triple-point isotherm, relaxation
// frequencies of oxygen (frO) and nitrogen (frN), then the classical plus
// rotational term and the two vibrational relaxation terms, in dB/m.
double gbs_air_absorption_db(double f_hz, double temp_c, double rh_pct, double pressure_atm) {
    if (!(f_hz > 0) || !(temp_c > -100 && temp_c < 100) || !(rh_pct >= 0 && rh_pct <= 100) || !(pressure_atm > 0))
        return NAN;
    const double T = temp_c + 273.15, tr = T / 293.15, pr = pressure_atm;
    const double psat_rel = std::pow(10.0, 4.6151 - 6.8346 * std::pow(273.16 / T, 1.261));
    const double h = rh_pct * psat_rel / pr;
    const double fro = pr * (24.0 + 4.04e4 * h * (0.02 + h) / (0.391 + h));
    const double frn = pr / std::sqrt(tr) * (9.0 + 280.0 * h * std::exp(-4.170 * (std::cbrt(1.0 / tr) - 1.0)));
    const double ff = f_hz * f_hz;
    const double classical = 1.84e-11 * std::sqrt(tr) / pr;
    const double vib = std::pow(tr, -2.5) * (0.01275 * std::exp(-2239.1 / T) * fro / (fro * fro + ff) +
                                             0.1068 * std::exp(-3352.0 / T) * frn / (frn * frn + ff));
    return 8.686 * ff * (classical + vib);
}

int gbs_create(gbs_ctx** out, int device, void* hip_stream) {
    if (!out) return GBS_E_INVALID;
    *out = nullptr;
    gbs_ctx* ctx = nullptr;
    try {
        ctx = new gbs_ctx;
    } catch (...) {
        return GBS_E_OOM;
    }
    int rc = guarded(ctx, [&]() {
        int n = 0;
        GBS_HIP(hipGetDeviceCount(&n));
        GBS_CHECK(device >= 0 && device < n, "device ordinal out of range");
        GBS_HIP(hipSetDevice(device));
        hipDeviceProp_t prop;
        GBS_HIP(hipGetDeviceProperties(&prop, device));
        ctx->device = device;
        ctx->n_cu = prop.multiProcessorCount;
        scratch_init(device);
        GBS_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->plan_words), 6 * sizeof(int64_t)));
        for (int i = 0; i < 2; ++i) GBS_HIP(hipEventCreateWithFlags(&ctx->planned[i], hipEventDisableTiming));
        ctx->stream = (hipStream_t)hip_stream;
        ctx->ws->stream = ctx->stream;
        return GBS_OK;
    });
    if (rc != GBS_OK) {
        for (int i = 0; i < 2; ++i)
            if (ctx->planned[i]) (void)hipEventDestroy(ctx->planned[i]);
        if (ctx->plan_words) (void)hipHostFree(ctx->plan_words);
        delete ctx;
        return rc;
    }
    *out = ctx;
    return GBS_OK;
}

void gbs_destroy(gbs_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->copy_stream) (void)hipStreamSynchronize(ctx->copy_stream);
    for (hipStream_t ps : ctx->pair_stream)
        if (ps) (void)hipStreamSynchronize(ps);
    ctx->ws.reset();
    for (int i = 0; i < 2; ++i) {
        if (ctx->pair_ready[i]) (void)hipEventDestroy(ctx->pair_ready[i]);
        if (ctx->pair_done[i]) (void)hipEventDestroy(ctx->pair_done[i]);
        if (ctx->pair_stream[i]) (void)hipStreamDestroy(ctx->pair_stream[i]);
        if (ctx->copied[i]) (void)hipEventDestroy(ctx->copied[i]);
        if (ctx->released[i]) (void)hipEventDestroy(ctx->released[i]);
        if (ctx->planned[i]) (void)hipEventDestroy(ctx->planned[i]);
    }
    if (ctx->plan_words) (void)hipHostFree(ctx->plan_words);
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    delete ctx;
}

int gbs_set_stream(gbs_ctx* ctx, void* hip_stream) {
    if (!ctx) return GBS_E_INVALID;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->ws->stream = ctx->stream;
    return GBS_OK;
}

const char* gbs_last_error(const gbs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int gbs_get_stats(const gbs_ctx* ctx, gbs_stats* out) {
    if (!ctx || !out) return GBS_E_INVALID;
    *out = ctx->stats;
    return GBS_OK;
}

int gbs_forward(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces, const double* rcv,
                int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps, const gbs_params* params,
                double* P, double* TL) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        Args a{rays, segs, faces, rcv, n_rcv, freqs, n_freq, eps, params};
        return forward_impl(ctx, *ctx->ws, a, P, TL, 0);
    });
}

int gbs_forward_noalloc(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                        const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                        const gbs_params* params, double* P, double* TL) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        if (params && (params->flags & GBS_FLAG_TABLE_HOST))
            throw GbsError(GBS_E_UNSUPPORTED, "gbs_forward_noalloc takes device tables only (a host table needs "
                                              "staging buffers); use gbs_forward");
        Workspace ws(scratch_base(ctx->device), kStaticScratchBytes);
        ws.stream = ctx->stream;
        Args a{rays, segs, faces, rcv, n_rcv, freqs, n_freq, eps, params};
        return forward_impl(ctx, ws, a, P, TL, 0);
    });
}

int gbs_backward(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces, const double* rcv,
                 int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps, const gbs_params* params,
                 const double* lambda, double* d_gamma, double* d_rcv, double* d_eps, double* d_eps_e2) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        Args a{rays, segs, faces, rcv, n_rcv, freqs, n_freq, eps, params};
        validate_host(a);
        GBS_CHECK(params->mode != GBS_MODE_F32, "the adjoint supports F64 and MIX");
        Workspace& ws = *ctx->ws;
        Planner pl(ctx, ws, a, 1);
        hipStream_t st = ctx->stream;
        const int n_jobs = pl.n_jobs;
        const int64_t n_out = (int64_t)n_jobs * n_rcv;
        GBS_CHECK(lambda || n_out == 0, "null lambda");
        const int32_t nf = faces->n_faces;
        double* Zf = ws.get<double>("Zf", 2 * std::max(nf, 1));
        double* dE = ws.get<double>("dE", std::max(2 * n_jobs, 1));   // d_eps, then d_eps_e2
        double* dRj = ws.get<double>("dR_job", std::max<int64_t>(3 * n_out, 1));
        fill(st, Zf, 2 * nf, 0.0);
        fill(st, dE, 2 * n_jobs, 0.0);
        fill(st, dRj, 3 * n_out, 0.0);
        gbs_stats stats{};
        stats.patch_rcv = 64;
        const bool timed = (params->flags & GBS_FLAG_TIME_KERNELS) != 0;
        if (n_out > 0 && segs->n_segs > 0) {
            pl.reset_status();
            // scales of the exact (order-independent) segment and face sums, from
            // sum |lambda| per job and, per pass, the coefficient-derivative bound
            double* l1 = ws.get<double>("lambda_l1", n_jobs);
            double* fscale = ws.get<double>("fixed_scales", 4);
            unsigned long long* bmax = ws.get<unsigned long long>("bmax", 1);
            // sum |lambda| per job over 64 pieces of the receivers, then the pieces in order
            const int pieces = 64;
            double* l1_part = ws.get<double>("lambda_l1_part", (int64_t)n_jobs * pieces);
            hipLaunchKernelGGL(k_lambda_l1, dim3(n_jobs, pieces), dim3(256), 0, st, lambda, n_rcv, l1_part,
                               pl.status);
            hipLaunchKernelGGL(k_lambda_l1_sum, dim3(blocks_for(n_jobs, 64)), dim3(64), 0, st, l1_part, n_jobs,
                               pieces, l1);
            GBS_HIP(hipGetLastError());
            pl.source_offsets();
            pl.make_passes();
            pl.plan_receivers(64);
            unsigned* ctr = ws.get<unsigned>("ctr", 1);
            for (size_t pi = 0; pi < pl.passes.size(); ++pi) {
                const PassRange& ps = pl.passes[pi];
                Planner::PassView v = pl.view(ps);
                fill(st, reinterpret_cast<double*>(bmax), 1, 0.0);
                Planner::Lists L = pl.build_lists(ps, v, (int)pi, bmax);
                stats.listed_pairs += L.total * 64;
                stats.n_items += L.n_items;
                const int64_t nseg = v.n_segs;
                hipLaunchKernelGGL(k_fixed_scales, dim3(1), dim3(64), 0, st, L.jobs, l1, n_jobs, nseg, bmax, fscale);
                Fixed* Sseg = ws.get<Fixed>("Sseg", 2 * std::max<int64_t>(nseg, 1));
                fill(st, reinterpret_cast<double*>(Sseg), 4 * nseg, 0.0);
                if (L.n_items > 0 && L.total > 0) {
                    const bool f64 = params->mode == GBS_MODE_F64, ab = pl.absorb();
                    auto kern = pl.aniso()
                                    ? (f64 ? (ab ? k_adjoint<12> : k_adjoint<8>) : (ab ? k_adjoint<13> : k_adjoint<9>))
                                    : (f64 ? (ab ? k_adjoint<4> : k_adjoint<0>) : (ab ? k_adjoint<5> : k_adjoint<1>));
                    double* part = ws.get<double>("adj_partial", L.work_cap * 64 * 3);
                    double* epart = ws.get<double>("eps_partial", 2 * L.work_cap);   // eps, then eps_e2
                    const int64_t grid = persistent_grid(ctx, (const void*)kern, L.work_cap);
                    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, st, ctr);
                    EventPair ev(timed);
                    ev.begin(st);
                    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kPairThreads), 0, st, L.jobs, L.work,
                                       L.n_work, pl.R.n_patch, ctr, L.lists, L.rec, L.frames, pl.R.rx, pl.R.ry,
                                       pl.R.rz, pl.R.r2, pl.R.perm, n_rcv, lambda, part, L.seg_perm, Sseg, fscale,
                                       epart, epart + L.work_cap);
                    GBS_HIP(hipGetLastError());
                    stats.ms_pairs += ev.end(st);
                    hipLaunchKernelGGL(k_reduce_adjoint, dim3(blocks_for((int64_t)L.n_items * 64, 256)), dim3(256), 0,
                                       st, L.jobs, L.item_wbase, L.item_wcount, L.n_items, pl.R.n_patch, pl.R.perm,
                                       n_rcv, part, dRj);
                    hipLaunchKernelGGL(k_reduce_eps, dim3(n_jobs), dim3(256), 0, st, L.item_wbase, L.item_wcount,
                                       pl.R.n_patch, epart, dE);
                    if (pl.aniso())
                        hipLaunchKernelGGL(k_reduce_eps, dim3(n_jobs), dim3(256), 0, st, L.item_wbase,
                                           L.item_wcount, pl.R.n_patch, epart + L.work_cap, dE + n_jobs);
                    GBS_HIP(hipGetLastError());
                }
                if (nf > 0 && nseg > 0) {
                    Fixed* Zfix = ws.get<Fixed>("Zfix", 2 * (int64_t)nf);
                    fill(st, reinterpret_cast<double*>(Zfix), 4 * (int64_t)nf, 0.0);
                    hipLaunchKernelGGL(k_face_scatter, dim3(blocks_for(nseg, 256)), dim3(256), 0, st, nseg,
                                       v.face_ptr, v.face_base, v.face_ids, nf, faces->gamma, v.ray_w, L.seg_ray,
                                       Sseg, fscale, Zfix);
                    hipLaunchKernelGGL(k_fixed_flush, dim3(blocks_for(2 * (int64_t)nf, 256)), dim3(256), 0, st, Zfix,
                                       2 * (int64_t)nf, fscale, Zf);
                    GBS_HIP(hipGetLastError());
                }
            }
            stats.n_chunks = (int32_t)pl.passes.size();
        }
        if (d_gamma && nf > 0)
            hipLaunchKernelGGL(k_dgamma, dim3(blocks_for(nf, 256)), dim3(256), 0, st, Zf, nf, d_gamma);
        if (d_rcv && n_rcv > 0)
            hipLaunchKernelGGL(k_sum_jobs, dim3(blocks_for(3 * n_rcv, 256)), dim3(256), 0, st, dRj, n_jobs, n_rcv,
                               d_rcv);
        if (d_eps && n_jobs > 0)
            GBS_HIP(hipMemcpyAsync(d_eps, dE, sizeof(double) * n_jobs, hipMemcpyDeviceToDevice, st));
        if (d_eps_e2 && n_jobs > 0 && params->eps_e2)
            GBS_HIP(hipMemcpyAsync(d_eps_e2, dE + n_jobs, sizeof(double) * n_jobs, hipMemcpyDeviceToDevice, st));
        GBS_HIP(hipGetLastError());
        int h_status = 0;
        if (pl.status) GBS_HIP(hipMemcpyAsync(&h_status, pl.status, sizeof(int), hipMemcpyDeviceToHost, st));
        GBS_HIP(hipStreamSynchronize(st));  // scratch reused by the next call
        check_status(h_status);
        stats.grid = ctx->stats.grid;
        stats.blocks_per_cu = ctx->stats.blocks_per_cu;
        ctx->stats = stats;
        return GBS_OK;
    });
}

int gbs_graph_create(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                     const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                     const gbs_params* params, double* P, double* TL, gbs_graph** out) {
    if (!ctx || !out) return GBS_E_INVALID;
    *out = nullptr;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        Args a{rays, segs, faces, rcv, n_rcv, freqs, n_freq, eps, params};
        validate_host(a);
        GBS_CHECK(!(params->flags & GBS_FLAG_COUNT_ACTIVE), "graphs do not count pairs");
        GBS_CHECK(ctx->stream != nullptr, "graph capture needs a non-null stream");
        std::unique_ptr<gbs_graph> g(new gbs_graph);
        g->ctx = ctx;
        Workspace& ws = *g->ws;
        ws.stream = ctx->stream;
        const int nr = pick_nr(ctx, params, n_rcv);
        Planner pl(ctx, ws, a, nr);
        hipStream_t st = ctx->stream;
        const int64_t n_out = (int64_t)pl.n_jobs * n_rcv;
        // plan every pass once (each pass keeps its own lists and work units);
        // a replay re-stages each pass's table (host tables: copies captured
        // from pinned memory), rebuilds its records and runs its pair kernel
        std::vector<Planner::Lists> Ls;
        const bool work = n_out > 0 && segs->n_segs > 0;
        int64_t cap = 0;
        if (work) {
            pl.reset_status();
            pl.source_offsets();
            pl.make_passes();
            pl.plan_receivers(64 * nr);
            for (size_t pi = 0; pi < pl.passes.size(); ++pi) {
                pl.tag = "#" + std::to_string(pi);
                Planner::PassView v = pl.view(pl.passes[pi]);
                Ls.push_back(pl.build_lists(pl.passes[pi], v, (int)pi));
                cap = std::max(cap, Ls.back().work_cap);
            }
        }
        double* partial = ws.get<double>("partial", std::max<int64_t>(cap, 1) * nr * 64 * 2);
        unsigned* ctr = ws.get<unsigned>("ctr", 1);
        GBS_HIP(hipStreamSynchronize(st));
        ws.frozen = true;
        GBS_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        try {
            fill(st, P, 2 * n_out, 0.0);
            for (size_t pi = 0; pi < Ls.size(); ++pi) {
                Planner::Lists L = Ls[pi];
                if (L.n_items == 0 || L.total == 0) continue;
                const Planner::PassView v = pl.view(pl.passes[pi]);
                // the pass's own planning buffers (named after its tag)
                const std::string t = "#" + std::to_string(pi);
                int32_t* seg_ray = ws.get<int32_t>("seg_ray" + t, v.n_segs);
                SegRec* rec = ws.get<SegRec>("rec" + t, v.n_segs);
                hipLaunchKernelGGL(k_seg2ray, dim3(blocks_for(v.n_rays, 256)), dim3(256), 0, st, v.ray_ptr, v.n_rays,
                                   pl.passes[pi].seg_begin, v.n_segs, seg_ray);
                // coefficients may change between replays: rebuild the records
                hipLaunchKernelGGL(k_records, dim3(blocks_for(v.n_segs, 256)), dim3(256), 0, st, v.n_segs, v.a, v.t,
                                   v.s0, v.lo, v.hi, v.face_ptr, v.face_base, v.face_ids, faces->n_faces,
                                   faces->gamma, v.ray_w, seg_ray, v.n_rays, pl.face_end_dev(),
                                   pl.face_end_host(pl.passes[pi]), rec, pl.status, nullptr);
                L.rec = rec;
                if (L.seg_perm) {   // into the spatial order planned at creation
                    SegRec* rs = ws.get<SegRec>("rec_sorted" + t, v.n_segs);
                    hipLaunchKernelGGL(k_permute_rec, dim3(blocks_for(v.n_segs, 256)), dim3(256), 0, st, v.n_segs,
                                       rec, L.seg_perm, rs);
                    L.rec = rs;
                }
                L.partial = partial;
                dispatch_pairs(params->mode, pl.absorb(), pl.aniso(), false, nr, ctx, st, L, pl.R, n_rcv, P, ctr, nullptr);
            }
            if (TL && n_out > 0)
                hipLaunchKernelGGL(k_tl, dim3(blocks_for(n_out, 256)), dim3(256), 0, st, P, n_out, TL);
        } catch (...) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(st, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            ws.frozen = false;
            throw;
        }
        GBS_HIP(hipStreamEndCapture(st, &g->graph));
        ws.frozen = false;
        GBS_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        *out = g.release();
        return GBS_OK;
    });
}

int gbs_graph_launch(gbs_graph* g) {
    if (!g || !g->exec) return GBS_E_INVALID;
    return guarded(g->ctx, [&]() {
        GBS_HIP(hipSetDevice(g->ctx->device));
        GBS_HIP(hipGraphLaunch(g->exec, g->ctx->stream));
        return GBS_OK;
    });
}

void gbs_graph_destroy(gbs_graph* g) {
    if (!g) return;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int gbs_impulse_response(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                         const double* rcv, int64_t n_rcv, double df, int32_t bin0, int32_t n_bins, const double* eps,
                         const double* window, const gbs_params* params, int32_t n_fft, int32_t n_t, double* h) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        GBS_CHECK(rays && segs && faces && params, "null struct argument");
        if (params->eps_e2)
            throw GbsError(GBS_E_UNSUPPORTED, "impulse responses support isotropic beams only");
        GBS_CHECK(std::isfinite(df) && df > 0, "df must be finite and > 0");
        GBS_CHECK(n_fft >= 64 && n_fft <= kIrMaxFft && (n_fft & (n_fft - 1)) == 0,
                  "n_fft must be a power of two in [64, 4096]");
        GBS_CHECK(bin0 >= 1 && n_bins >= 1 && (int64_t)bin0 + n_bins <= n_fft / 2,
                  "bins must satisfy 1 <= bin0 and bin0 + n_bins <= n_fft / 2");
        GBS_CHECK(n_t >= 1 && n_t <= n_fft, "n_t must be in [1, n_fft]");
        GBS_CHECK(n_rcv >= 0 && rays->n_src >= 0, "negative size");
        const int n_src = rays->n_src;
        const int64_t rows = (int64_t)n_src * n_rcv;
        GBS_CHECK(rows == 0 || (eps && h), "null eps or h");
        GBS_CHECK(rows <= INT32_MAX, "too many (source, receiver) rows");
        hipStream_t st = ctx->stream;
        Workspace& ws = *ctx->ws;
        const int64_t nj = (int64_t)n_src * n_bins;
        std::vector<double> h_eps(nj), h_alpha(params->alpha ? nj : 0), h_win(window ? n_bins : 0);
        if (nj > 0) {
            GBS_HIP(hipMemcpyAsync(h_eps.data(), eps, sizeof(double) * nj, hipMemcpyDeviceToHost, st));
            if (params->alpha)
                GBS_HIP(hipMemcpyAsync(h_alpha.data(), params->alpha, sizeof(double) * nj, hipMemcpyDeviceToHost,
                                       st));
            if (window)
                GBS_HIP(hipMemcpyAsync(h_win.data(), window, sizeof(double) * n_bins, hipMemcpyDeviceToHost, st));
            GBS_HIP(hipStreamSynchronize(st));
        }
        for (double w : h_win) GBS_CHECK(std::isfinite(w), "window must be finite");
        if (rows == 0) return GBS_OK;
        int log2n = 0;
        while ((1 << log2n) < n_fft) ++log2n;
        double2* spec = ws.get<double2>("ir_spec", (size_t)rows * n_fft);
        fill(st, reinterpret_cast<double*>(spec), 2 * rows * n_fft, 0.0);
        double2* tw = ws.get<double2>("ir_tw", n_fft / 2);
        hipLaunchKernelGGL(k_ir_twiddles, dim3(blocks_for(n_fft / 2, 256)), dim3(256), 0, st, n_fft, tw);
        GBS_HIP(hipGetLastError());
        // the spectrum, up to kMaxBands bins per forward call
        std::vector<double> fc, ec, ac;
        for (int b0 = 0; b0 < n_bins; b0 += kMaxBands) {
            const int nb = std::min(kMaxBands, n_bins - b0);
            fc.resize(nb);
            ec.resize((size_t)n_src * nb);
            ac.resize(params->alpha ? (size_t)n_src * nb : 0);
            for (int b = 0; b < nb; ++b) fc[b] = (double)(bin0 + b0 + b) * df;
            for (int s = 0; s < n_src; ++s)
                for (int b = 0; b < nb; ++b) {
                    ec[(size_t)s * nb + b] = h_eps[(size_t)s * n_bins + b0 + b];
                    if (params->alpha) ac[(size_t)s * nb + b] = h_alpha[(size_t)s * n_bins + b0 + b];
                }
            double* d_f = ws.get<double>("ir_freqs", kMaxBands);
            double* d_e = ws.get<double>("ir_eps", (size_t)n_src * kMaxBands);
            double* d_a = ws.get<double>("ir_alpha", (size_t)n_src * kMaxBands);
            GBS_HIP(hipMemcpyAsync(d_f, fc.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
            GBS_HIP(hipMemcpyAsync(d_e, ec.data(), sizeof(double) * ec.size(), hipMemcpyHostToDevice, st));
            if (params->alpha)
                GBS_HIP(hipMemcpyAsync(d_a, ac.data(), sizeof(double) * ac.size(), hipMemcpyHostToDevice, st));
            gbs_params pc = *params;
            pc.alpha = params->alpha ? d_a : nullptr;
            double* Pc = ws.get<double>("ir_P", (size_t)2 * n_src * nb * n_rcv);
            Args a{rays, segs, faces, rcv, n_rcv, d_f, nb, d_e, &pc};
            forward_impl(ctx, ws, a, Pc, nullptr, 0);
            const int64_t n_sc = (int64_t)n_src * nb * n_rcv;
            hipLaunchKernelGGL(k_ir_scatter, dim3(blocks_for(n_sc, 256)), dim3(256), 0, st, Pc, n_src, nb, n_rcv,
                               bin0 + b0, window, b0, n_fft, spec);
            GBS_HIP(hipGetLastError());
            GBS_HIP(hipStreamSynchronize(st));      // the host chunk arrays are rewritten next
        }
        hipLaunchKernelGGL(k_ir_fft, dim3((unsigned)rows), dim3(256), sizeof(double2) * n_fft, st, spec, n_fft,
                           log2n, tw, 2.0 * df, n_t, h);
        GBS_HIP(hipGetLastError());
        return GBS_OK;
    });
}

int gbs_trace_count(gbs_ctx* ctx, const gbs_scene* scene, const gbs_fan* fan, int64_t* n_segs,
                    int64_t* n_face_ids, int64_t* token) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_CHECK(n_segs && n_face_ids, "n_segs and n_face_ids must be non-null");
        GBS_HIP(hipSetDevice(ctx->device));
        const auto r = trace_impl(ctx, scene, fan, 0, 0, nullptr);
        *n_segs = r.first;
        *n_face_ids = r.second;
        if (token) *token = ctx->trace_token;
        return GBS_OK;
    });
}

int gbs_trace(gbs_ctx* ctx, const gbs_scene* scene, const gbs_fan* fan, int64_t token, int64_t cap_segs,
              int64_t cap_face_ids, int64_t* ray_ptr, double* seg_a, double* seg_t, double* seg_s0, double* seg_lo,
              double* seg_hi, int64_t* face_ptr, int32_t* face_ids, double* seg_e1, int64_t* n_segs,
              int64_t* n_face_ids) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_CHECK(ray_ptr, "ray_ptr must be non-null");
        GBS_HIP(hipSetDevice(ctx->device));
        const TraceOut o{ray_ptr, seg_a, seg_t, seg_s0, seg_lo, seg_hi, face_ptr, face_ids, seg_e1};
        const auto r = trace_impl(ctx, scene, fan, cap_segs, cap_face_ids, &o, token);
        if (n_segs) *n_segs = r.first;
        if (n_face_ids) *n_face_ids = r.second;
        return GBS_OK;
    });
}

int gbs_autotune(gbs_ctx* ctx, const gbs_rays* rays, const gbs_segs* segs, const gbs_faces* faces,
                 const double* rcv, int64_t n_rcv, const double* freqs, int32_t n_freq, const double* eps,
                 const gbs_params* params, double* P, int32_t* rcv_per_lane, int32_t* work_chunk) {
    if (!ctx) return GBS_E_INVALID;
    return guarded(ctx, [&]() {
        GBS_HIP(hipSetDevice(ctx->device));
        Args a{rays, segs, faces, rcv, n_rcv, freqs, n_freq, eps, params};
        validate_host(a);
        EventPair ev(true);
        float best = 1e30f;
        int best_nr = 1, best_chunk = kWorkChunk;
        for (int nr : {1, 2, 4})
            for (int chunk : {1024, 2048, 4096}) {
                forward_impl(ctx, *ctx->ws, a, P, nullptr, nr, chunk);  // warm-up and plan
                float ms = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {                       // best of two
                    ev.begin(ctx->stream);
                    forward_impl(ctx, *ctx->ws, a, P, nullptr, nr, chunk);
                    ms = std::min(ms, (float)ev.end(ctx->stream));
                }
                if (ms < best) {
                    best = ms;
                    best_nr = nr;
                    best_chunk = chunk;
                }
            }
        ctx->tuned_nr[params->mode] = best_nr;
        ctx->tuned_chunk[params->mode] = best_chunk;
        if (rcv_per_lane) *rcv_per_lane = best_nr;
        if (work_chunk) *work_chunk = best_chunk;
        return GBS_OK;
    });
}

}  // extern "C"
