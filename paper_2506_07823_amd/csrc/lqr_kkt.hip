// lqr_kkt.hip -- host side of the C ABI declared in include/lqr_kkt.h.
//
// Builds the launch plan (tree shapes, workspace layout), validates the
// arguments, and enqueues the kernels of kernels.hpp on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/lqr_kkt.h"
#include "pack.hpp"
#include "qpdata.hpp"
#include "runs.hpp"
#include "sqp.hpp"

using namespace lqr;

// Workspace of lqr_kkt_solve_noalloc: one array of kNoAllocBytes in each
// GPU's copy of the library's device code, held until the process ends.  In
// host code its name is only a stand-in: the device address of each GPU's
// copy is looked up once per device (lqr_create) and kept in g_scratch.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

thread_local std::string g_err;
thread_local lqr::Timer* g_timer = nullptr;

lqr::Timer*& lqr::current_timer() { return g_timer; }

int lqr::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

namespace lqr {
LQR_DECLARE_RUNS(1)
LQR_DECLARE_RUNS(2)
LQR_DECLARE_RUNS(3)
LQR_DECLARE_RUNS(4)
LQR_DECLARE_RUNS(5)
LQR_DECLARE_RUNS(6)
LQR_DECLARE_RUNS(8)
LQR_DECLARE_RUNS(32)
}  // namespace lqr

namespace {

// padded-order class: TS = ceil(max(n, m) / 8) for the wavefront engine
// (orders up to 64), the large-block engine (kBigTS) up to kMaxDim
constexpr int kTS[] = {1, 2, 3, 4, 5, 6, 8};
constexpr int kMaxDim = 256;
int pick_ts(int n, int m) {
    const int d = n > m ? n : m;
    for (int ts : kTS)
        if (8 * ts >= d) return ts;
    return d <= kMaxDim ? kBigTS : 0;
}

// Mapping choices the autotuner may override (0 / -1: the default rule)
struct Tuning {
    int engine = 0;     // 1: wavefront tiles, 2: matrix-core workgroups
    int fused = -1;     // vector passes level by level 0, per instance 1; 2: whole solve in one launch
    int big_grid = 0;   // workgroups (scratch slots) of a matrix-core task launch
    int split = 0;      // reverse scan: 0 balanced tree, 1 split, 2 chunked (wavefront engine)
    int chunk = 0;      // chunked schedule: chunk length (>= 1)
    int sweep = 0;      // chunked schedule: leaves of the sequential sweep (>= 1, the terminal included)
    int fwd_seq = 0;    // 1: sequential forward and refinement vector passes
    int streams = 0;    // 2..kMaxParts: the batch in that many contiguous parts, one stream each
};

// Most parts of a batch split over streams (part 0 on the caller's stream,
// the others on the handle's side streams)
constexpr int kMaxParts = 4;

int pick_ts(int n, int m, const Tuning* t) {
    const int ts = pick_ts(n, m);
    if (t && t->engine == 2 && ts != 0) return kBigTS;
    return ts;
}
// workgroups (= scratch slots) of a large-block task launch
constexpr int kBigGrid = 512;
// slots of the FP64 redo of marked instances
constexpr int kRedoSlots = 128;

Plan make_plan(int64_t batch, int N, int n, int m, size_t esize, const lqr_opts& o, const Tuning* tun = nullptr) {
    Plan p;
    std::memset(&p, 0, sizeof p);
    p.batch = batch;
    plan_records(p, N, n, m);
    p.cond_thr = o.cond_threshold;
    p.refine_tol = o.refine_tol;
    p.active = nullptr;
    // vector-only passes level by level (one workgroup per tree node or
    // stage); the per-instance form (one workgroup walks an instance) is a
    // mapping the autotuner may pick instead
    p.fused = 0;
    p.fallback = esize == 4 ? o.fallback : 0;   // the FP64 path has nothing to fall back to
    if (tun && tun->fused >= 0) p.fused = tun->fused;
    const bool big = pick_ts(n, m, tun) == kBigTS;
    p.sched = 0;
    if (tun && tun->split && p.fused != 2 && !big) {
        if (tun->split == 1) {
            // split: the tree over the largest power of two of leaves below
            // N + 1 (every tree level above the leaves has a node past it),
            // the rest by the sequential sweep
            p.sched = 1;
            p.tail = 1 << (p.rt.nlev - 2);
        } else {
            // chunked: `sweep` leaves swept sequentially, chunks of `chunk`
            // leaves over the rest
            p.sched = 2;
            const int sweep = std::min(std::max(tun->sweep, 1), N + 1);
            p.tail = N + 1 - sweep;
            p.chunk = std::max(tun->chunk, 1);
            p.nchunk = (p.tail + p.chunk - 1) / p.chunk;
        }
    }
    p.fwdseq = tun && tun->fwd_seq && p.fused != 2 ? 1 : 0;
    // the chunked schedule's sweeps combine each leaf through its rank-m factor
    p.leafv = p.sched == 2 && p.o_V >= 0 ? 1 : 0;
    // chunk length 1 and a sweep of the terminal element only: every leaf
    // is combined in the leaf form, none reads its C
    p.noC = p.leafv && p.chunk == 1 && p.tail == N ? 1 : 0;
    // and then the sweep builds each leaf itself where V' and W_M fit the
    // two halves of one LDS slot (2 ceil(m/8) <= the tile's blocks)
    {
        const int lw = m <= 8 ? 1 : 2, ts = pick_ts(n, m, tun);
        p.fuse_elem = p.noC && ts != kBigTS && 2 * lw <= ts ? 1 : 0;
    }
    if (big) {
        if (p.fused == 2) p.fused = 1;   // the one-launch solve is a wavefront-engine form
        const int64_t d = n > m ? n : m;
        p.scr_elems = align_up(8 * d * d + 64 * d, 64);
        const int64_t most = batch * (N + 1);
        const int64_t g = tun && tun->big_grid > 0 ? tun->big_grid : kBigGrid;
        p.big_grid = (int)(most < g ? most : g);
    }
    return p;
}

// Plan of the FP64 redo slots: per slot P_k, p_k (suffix area by stage), K_k,
// k_k in FP64 (plus, for the large-block engine, an FP64 scratch area of one
// element block per slot after all slots)
Plan make_redo_plan(const Plan& p, bool big, int64_t& slots, size_t& bytes) {
    Plan r = p;
    r.active = nullptr;
    redo_records(r);
    slots = std::min<int64_t>(p.batch, kRedoSlots);
    r.big_grid = (int)slots;
    bytes = (size_t)(slots * r.stride * 8);
    if (big) {
        r.o_scr = (int64_t)align_up((int64_t)bytes, 256);
        bytes = (size_t)r.o_scr + (size_t)(slots * p.scr_elems * 8);
    }
    bytes = (size_t)align_up((int64_t)bytes, 256);
    return r;
}

struct Layout {
    size_t main_bytes, int_off, dbl_off, scr_off, redo_off, total;
};

// per-instance records | int32 refinement flags | FP64 partial sums |
// large-block scratch (one slot per workgroup) | FP64 redo slots
Layout layout(const Plan& p, size_t esize) {
    Layout l;
    l.main_bytes = (size_t)align_up((int64_t)(p.batch * p.stride * (int64_t)esize), 256);
    l.int_off = l.main_bytes;
    l.dbl_off = l.int_off + (size_t)align_up(p.batch * 4, 256);
    l.scr_off = l.dbl_off + (size_t)align_up((p.batch * p.dstride + p.batch) * 8, 256);
    l.redo_off = l.scr_off + (size_t)align_up((int64_t)p.big_grid * p.scr_elems * (int64_t)esize, 256);
    l.total = l.redo_off;
    if (p.fallback) {
        int64_t slots;
        size_t rb;
        make_redo_plan(p, p.big_grid > 0, slots, rb);
        l.total += rb;
    }
    return l;
}

bool aligned(const void* ptr, size_t a) { return ((uintptr_t)ptr % a) == 0; }

// A batch split over streams: `count` contiguous parts of `size` instances
// (the last may be smaller), each with a workspace slice of `bytes`.
struct Parts {
    int count;
    int64_t size;
    size_t bytes;
};

Parts parts_of(int64_t batch, int N, int n, int m, size_t es, const lqr_opts& o, const Tuning* tun) {
    Parts r;
    int k = tun && tun->streams > 1 ? std::min(tun->streams, kMaxParts) : 1;
    if (o.method == LQR_METHOD_SEQ_RICCATI || k > batch) k = 1;
    r.size = (batch + k - 1) / k;
    r.count = (int)((batch + r.size - 1) / r.size);
    // slices always hold the FP64 redo area, so that their offsets do not
    // depend on the call's options (a re-solve or a factor read-back of
    // this shape finds the records where the solve left them)
    lqr_opts of = o;
    of.fallback = 1;
    r.bytes = (size_t)align_up((int64_t)layout(make_plan(r.size, N, n, m, es, of, tun), es).total, 256);
    return r;
}

// workspace bytes of a solve (every part's slice)
size_t solve_bytes(int64_t batch, int N, int n, int m, size_t es, const lqr_opts& o, const Tuning* tun) {
    const Parts pt = parts_of(batch, N, n, m, es, o, tun);
    if (pt.count == 1) return layout(make_plan(batch, N, n, m, es, o, tun), es).total;
    return pt.bytes * (size_t)pt.count;
}

int check_dims(int64_t batch, int N, int n, int m) {
    if (batch < 1) return fail(LQR_EINVAL, "batch must be >= 1 (got %lld)", (long long)batch);
    if (N < 1 || n < 1 || m < 1) return fail(LQR_EINVAL, "N, n, m must be >= 1 (got %d, %d, %d)", N, n, m);
    if (pick_ts(n, m) == 0)
        return fail(LQR_EUNSUPPORTED, "n=%d m=%d exceed the built shape classes (<= %d)", n, m, kMaxDim);
    if (N + 1 > (1 << (LQR_MAXLEV - 2))) return fail(LQR_EINVAL, "N=%d too large", N);
    const int64_t tasks = batch * (int64_t)(N + 1);
    if (tasks > (int64_t)0x7fffffff) return fail(LQR_EINVAL, "batch*(N+1) exceeds the grid limit");
    return LQR_OK;
}

// the chunked schedule keeps its aggregates in records of the tree levels
// above the leaves (two per chunk of two or more leaves): they must exist
bool sched_fits(const Plan& p) {
    if (p.sched != 2) return true;
    for (int c = 0; c < p.nchunk; ++c) {
        const int c0 = c * p.chunk, len = std::min(c0 + p.chunk, p.tail) - c0;
        if (len >= 2 && p.rt.off[1] + 2 * c + (len >= 3 ? 1 : 0) >= p.rt.total) return false;
    }
    return true;
}

// internal method code of lqr_kkt_resolve
constexpr int kResolve = -1;

template <typename S>
int dispatch(int ts, int method, const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws,
             const Ctx& cx, int refine, double* resid_out, const Warm<S>& warm) {
#define LQR_CASE(TSV)                                                                    \
    case TSV:                                                                            \
        return method == LQR_METHOD_SCAN                                                 \
                   ? run_scan<S, TSV>(p, s, in, out, ws, cx, refine, resid_out, warm)    \
                   : method == kResolve ? run_resolve<S, TSV>(p, s, in, out, ws, cx, refine, resid_out) \
                                        : run_plain<S, TSV>(p, s, in, out, ws, cx, resid_out);
    switch (ts) {
        LQR_CASE(1) LQR_CASE(2) LQR_CASE(3) LQR_CASE(4) LQR_CASE(5) LQR_CASE(6) LQR_CASE(8) LQR_CASE(32)
        default: return fail(LQR_EUNSUPPORTED, "no shape class for TS=%d", ts);
    }
#undef LQR_CASE
}

template <typename S>
int dispatch_resid(int ts, const Plan& p, hipStream_t s, const In<S>& in, const S* x, const S* u,
                   const S* lam, S* ws, double* dws, double* rel) {
#define LQR_CASE(TSV) \
    case TSV: return run_resid<S, TSV>(p, s, in, x, u, lam, ws, dws, rel);
    switch (ts) {
        LQR_CASE(1) LQR_CASE(2) LQR_CASE(3) LQR_CASE(4) LQR_CASE(5) LQR_CASE(6) LQR_CASE(8) LQR_CASE(32)
        default: return fail(LQR_EUNSUPPORTED, "no shape class for TS=%d", ts);
    }
#undef LQR_CASE
}

}  // namespace

namespace {
const char* const kFamNames[F_COUNT] = {
    "clear", "element", "up", "root", "down", "policy", "fwd_up", "fwd_root", "fwd_down", "recover", "residual",
    "ref_d", "bwd_up", "bwd_root", "bwd_down", "ref_kff", "fwd_up_vec", "recover_add", "reduce", "plain_riccati",
    "fwd_inst", "refine_inst", "warm_copy", "ragged_pack", "fused_solve", "tail_sweep", "tail_root",
    "tail_sweep_up0", "chunk_up", "chunk_mid", "chunk_down", "fwd_seq", "refine_seq", "fp64_redo", "mark_redo", "ragged_solve", "resolve", "sqp"};

// Per-handle launch timer: two HIP events around every launch, read back by
// lqr_timing_report.
struct EventTimer final : lqr::Timer {
    struct Rec { int fam; hipEvent_t a, b; double flops, bytes, flops_min; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    Rec cur{};
    void before(hipStream_t s, int fam, double flops, double bytes, double flops_min) override {
        cur = Rec{fam, get(), get(), flops, bytes, flops_min};
        if (cur.a) (void)hipEventRecord(cur.a, s);
    }
    void after(hipStream_t s) override {
        if (cur.b) (void)hipEventRecord(cur.b, s);
        if (cur.a && cur.b) recs.push_back(cur);
    }
    ~EventTimer() override {
        for (auto& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

struct TimerScope {
    explicit TimerScope(lqr::Timer* t) { g_timer = t; }
    ~TimerScope() { g_timer = nullptr; }
};
}  // namespace

struct lqr_handle_s {
    int device;
    bool timing = false;
    EventTimer timer;
    // mappings chosen by lqr_autotune / lqr_set_tuning, per (batch, N, n, m,
    // dtype), and per shape bucket (batch and N rounded up to powers of two:
    // what the tuning cache file holds)
    std::map<std::tuple<int64_t, int, int, int, int>, Tuning> tuned, cached;
    const Tuning* find(int64_t batch, int N, int n, int m, int dtype) const;
    // side streams of a batch split over streams (non-blocking, default
    // priority) and the events that fork them from the caller's stream and
    // join them back; made with the handle, so that a solve under stream
    // capture creates nothing
    hipStream_t side[kMaxParts - 1] = {};
    hipEvent_t fork = nullptr, join[kMaxParts - 1] = {};
    ~lqr_handle_s() {
        for (hipStream_t st : side)
            if (st) (void)hipStreamDestroy(st);
        for (hipEvent_t ev : join)
            if (ev) (void)hipEventDestroy(ev);
        if (fork) (void)hipEventDestroy(fork);
    }
};

extern "C" {

void lqr_opts_default(lqr_opts* o, int32_t dtype) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->dtype = dtype;
    o->method = LQR_METHOD_SCAN;
    o->refine_sweeps = dtype == LQR_F32 ? 1 : 0;
    o->fallback = 1;
    o->cond_threshold = 1e6;
    o->refine_tol = 1e-6;
    o->resid_out = nullptr;
    o->sync_status = 0;
}

int lqr_create(lqr_handle_t* h, int device) {
    if (!h) return fail(LQR_EINVAL, "null handle pointer");
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(LQR_EINVAL, "device %d out of range (%d devices)", device, count);
    if (device >= kMaxDevices) return fail(LQR_EINVAL, "device %d beyond the %d this library tracks", device, kMaxDevices);
    {
        // device address of this GPU's no-allocation workspace (once per device)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            int prev = 0;
            HIPCHK(hipGetDevice(&prev));
            HIPCHK(hipSetDevice(device));
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            HIPCHK(hipSetDevice(prev));
            if (e != hipSuccess)
                return fail(LQR_EDEVICE, "hipGetSymbolAddress of the no-allocation workspace: %s", hipGetErrorString(e));
            g_scratch[device] = ptr;
        }
    }
    lqr_handle_s* hh = new lqr_handle_s;
    hh->device = device;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    for (int i = 0; i < kMaxParts - 1 && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&hh->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&hh->join[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&hh->fork, hipEventDisableTiming);
    (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        delete hh;
        return fail(LQR_EDEVICE, "creating the handle's side streams: %s", hipGetErrorString(e));
    }
    *h = hh;
    return LQR_OK;
}

int lqr_destroy(lqr_handle_t h) {
    delete h;
    return LQR_OK;
}

int lqr_max_dim(void) { return kMaxDim; }

const char* lqr_last_error(void) { return g_err.c_str(); }

int lqr_workspace_size(lqr_handle_t h, int64_t batch, int N, int n, int m, const lqr_opts* opts,
                       size_t* bytes) {
    if (!bytes) return fail(LQR_EINVAL, "null output pointer");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    LCHK(check_dims(batch, N, n, m));
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    const Tuning* tun = h ? h->find(batch, N, n, m, o.dtype) : nullptr;
    *bytes = solve_bytes(batch, N, n, m, es, o, tun);
    return LQR_OK;
}

}  // extern "C"

namespace {
// the buffers of a call beside the records, carved from the workspace
Ctx make_ctx(const Plan& p, const Layout& lay, char* wsb, bool big) {
    Ctx cx;
    cx.active = (int32_t*)(wsb + lay.int_off);
    cx.dws = (double*)(wsb + lay.dbl_off);
    cx.ws64 = nullptr;
    cx.redo_grid = 0;
    std::memset(&cx.rp, 0, sizeof cx.rp);
    if (p.fallback) {
        int64_t slots;
        size_t rb;
        cx.rp = make_redo_plan(p, big, slots, rb);
        cx.ws64 = (double*)(wsb + lay.redo_off);
        cx.redo_grid = (int)slots;
    }
    return cx;
}

// LQR_ENUMERIC check of a call with opts.sync_status: wait for the stream
// and read the status words back
int sync_status_check(hipStream_t s, const int32_t* status, int64_t batch) {
    std::vector<int32_t> st((size_t)batch);
    HIPCHK(hipMemcpyAsync(st.data(), status, sizeof(int32_t) * (size_t)batch, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t bad = 0, first = -1;
    for (int64_t b = 0; b < batch; ++b)
        if (st[(size_t)b] & ~LQR_ST_FP64_FALLBACK) {
            if (first < 0) first = b;
            ++bad;
        }
    if (bad)
        return fail(LQR_ENUMERIC, "%lld instance(s) failed (first: instance %lld, status %d)", (long long)bad,
                    (long long)first, st[(size_t)first]);
    return LQR_OK;
}

int solve_impl(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, const void* A, const void* B,
               const void* c, const void* Q, const void* R, const void* M, const void* q, const void* r,
               const void* x0, void* x, void* u, void* lam, int32_t* status, void* workspace,
               size_t workspace_bytes, const lqr_opts& o, const Tuning* tun) {
    LCHK(check_dims(batch, N, n, m));
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    if (o.method != LQR_METHOD_SCAN && o.method != LQR_METHOD_SEQ_RICCATI && o.method != kResolve)
        return fail(LQR_EINVAL, "bad method %d", o.method);
    if (o.refine_sweeps < 0 || o.refine_sweeps > 4) return fail(LQR_EINVAL, "refine_sweeps must be in 0..4");
    if (!(o.refine_tol > 0.0)) return fail(LQR_EINVAL, "refine_tol must be > 0");
    if (!(o.cond_threshold > 1.0)) return fail(LQR_EINVAL, "cond_threshold must be > 1");
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    const void* ins[] = {A, B, c, Q, R, M, q, r, x0};
    const char* names[] = {"A", "B", "c", "Q", "R", "M", "q", "r", "x0"};
    for (int i = 0; i < 9; ++i) {
        if (!ins[i]) return fail(LQR_EINVAL, "null input %s", names[i]);
        if (!aligned(ins[i], es)) return fail(LQR_EINVAL, "input %s not aligned to %zu bytes", names[i], es);
    }
    if (!x || !u || !lam || !status || !workspace) return fail(LQR_EINVAL, "null output, status or workspace");
    if (!aligned(x, es) || !aligned(u, es) || !aligned(lam, es) || !aligned(status, 4))
        return fail(LQR_EINVAL, "misaligned output");
    if (!aligned(workspace, 256)) return fail(LQR_EINVAL, "workspace must be 256-byte aligned");
    if (o.resid_out && !aligned(o.resid_out, 8)) return fail(LQR_EINVAL, "misaligned resid_out");
    const bool has_warm = o.warm_x || o.warm_u || o.warm_lam;
    if (has_warm) {
        if (!o.warm_x || !o.warm_u || !o.warm_lam) return fail(LQR_EINVAL, "warm start needs x, u and lam");
        if (!aligned(o.warm_x, es) || !aligned(o.warm_u, es) || !aligned(o.warm_lam, es))
            return fail(LQR_EINVAL, "misaligned warm start");
    }
    if (!sched_fits(make_plan(1, N, n, m, es, o, tun)))
        return fail(LQR_EINVAL, "chunked schedule does not fit the tree records of N=%d", N);
    const Parts pt = parts_of(batch, N, n, m, es, o, tun);
    const size_t need = solve_bytes(batch, N, n, m, es, o, tun);
    if (workspace_bytes < need)
        return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, need);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int ts = pick_ts(n, m, tun);
    const int refine = o.method != LQR_METHOD_SEQ_RICCATI ? o.refine_sweeps : 0;
    // instances [b0, b0 + cnt) on stream sj with the workspace at wsb
    auto run_part = [&](int64_t b0, int64_t cnt, hipStream_t sj, char* wsb) -> int {
        Plan p = make_plan(cnt, N, n, m, es, o, tun);
        const Layout lay = layout(p, es);
        p.o_scr = (int64_t)lay.scr_off;
        const Ctx cx = make_ctx(p, lay, wsb, ts == kBigTS);
        const int64_t sN = b0 * N, sN1 = b0 * (N + 1);
        double* rout = o.resid_out ? o.resid_out + b0 : nullptr;
        if (o.dtype == LQR_F32) {
            using F = float;
            In<F> in{(const F*)A + sN * n * n, (const F*)B + sN * n * m, (const F*)c + sN * n,
                     (const F*)Q + sN1 * n * n, (const F*)R + sN * m * m, (const F*)M + sN * n * m,
                     (const F*)q + sN1 * n, (const F*)r + sN * m, (const F*)x0 + b0 * n};
            Out<F> out{(F*)x + sN1 * n, (F*)u + sN * m, (F*)lam + sN1 * n, status + b0};
            const Warm<F> warm{o.warm_x ? (const F*)o.warm_x + sN1 * n : nullptr,
                               o.warm_u ? (const F*)o.warm_u + sN * m : nullptr,
                               o.warm_lam ? (const F*)o.warm_lam + sN1 * n : nullptr};
            return dispatch<F>(ts, o.method, p, sj, in, out, (F*)wsb, cx, refine, rout, warm);
        } else {
            using F = double;
            In<F> in{(const F*)A + sN * n * n, (const F*)B + sN * n * m, (const F*)c + sN * n,
                     (const F*)Q + sN1 * n * n, (const F*)R + sN * m * m, (const F*)M + sN * n * m,
                     (const F*)q + sN1 * n, (const F*)r + sN * m, (const F*)x0 + b0 * n};
            Out<F> out{(F*)x + sN1 * n, (F*)u + sN * m, (F*)lam + sN1 * n, status + b0};
            const Warm<F> warm{o.warm_x ? (const F*)o.warm_x + sN1 * n : nullptr,
                               o.warm_u ? (const F*)o.warm_u + sN * m : nullptr,
                               o.warm_lam ? (const F*)o.warm_lam + sN1 * n : nullptr};
            return dispatch<F>(ts, o.method, p, sj, in, out, (F*)wsb, cx, refine, rout, warm);
        }
    };
    int rc = LQR_OK;
    {
        TimerScope ts_scope(h->timing ? &h->timer : nullptr);
        if (pt.count == 1) {
            rc = run_part(0, batch, s, (char*)workspace);
        } else {
            // fork: every side stream waits for the work queued so far on
            // the caller's stream; join: the caller's stream waits for every
            // side stream that was forked (also after an error, so that no
            // side stream is left outside a stream capture)
            HIPCHK(hipEventRecord(h->fork, s));
            int forked = 0;
            for (int j = 0; j < pt.count && rc == LQR_OK; ++j) {
                hipStream_t sj = s;
                if (j > 0) {
                    if (hipStreamWaitEvent(h->side[j - 1], h->fork, 0) != hipSuccess) {
                        rc = fail(LQR_EDEVICE, "forking side stream %d failed", j);
                        break;
                    }
                    forked = j;
                    sj = h->side[j - 1];
                }
                const int64_t b0 = j * pt.size;
                rc = run_part(b0, std::min(pt.size, batch - b0), sj, (char*)workspace + (size_t)j * pt.bytes);
            }
            for (int j = 1; j <= forked; ++j) {
                const hipError_t e1 = hipEventRecord(h->join[j - 1], h->side[j - 1]);
                const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s, h->join[j - 1], 0) : e1;
                if (e2 != hipSuccess && rc == LQR_OK) rc = fail(LQR_EDEVICE, "joining side stream %d failed", j);
            }
        }
    }
    if (rc != LQR_OK || !o.sync_status) return rc;
    return sync_status_check(s, status, batch);
}
}  // namespace

extern "C" {

int lqr_kkt_solve(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, const void* A,
                  const void* B, const void* c, const void* Q, const void* R, const void* M, const void* q,
                  const void* r, const void* x0, void* x, void* u, void* lam, int32_t* status,
                  void* workspace, size_t workspace_bytes, const lqr_opts* opts) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.method == kResolve) return fail(LQR_EINVAL, "bad method %d", o.method);
    return solve_impl(h, stream, batch, N, n, m, A, B, c, Q, R, M, q, r, x0, x, u, lam, status, workspace,
                      workspace_bytes, o, h->find(batch, N, n, m, o.dtype));
}

int lqr_kkt_solve_noalloc(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, const void* A,
                          const void* B, const void* c, const void* Q, const void* R, const void* M, const void* q,
                          const void* r, const void* x0, void* x, void* u, void* lam, int32_t* status,
                          const lqr_opts* opts) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.sync_status) return fail(LQR_EINVAL, "sync_status is not available without allocation");
    if (o.method == kResolve) return fail(LQR_EINVAL, "bad method %d", o.method);
    void* ws = g_scratch[h->device];
    if (!ws) return fail(LQR_EDEVICE, "no-allocation workspace of device %d not set up", h->device);
    LCHK(check_dims(batch, N, n, m));
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const Tuning* tun = h->find(batch, N, n, m, o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    const size_t need = solve_bytes(batch, N, n, m, es, o, tun);
    if (need > kNoAllocBytes)
        return fail(LQR_ENOMEM, "this solve needs %zu bytes of workspace, more than the %zu of the no-allocation "
                    "workspace; use lqr_kkt_solve with a caller workspace", need, kNoAllocBytes);
    return solve_impl(h, stream, batch, N, n, m, A, B, c, Q, R, M, q, r, x0, x, u, lam, status, ws, kNoAllocBytes,
                      o, tun);
}

int lqr_kkt_resolve(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, const void* A, const void* B,
                    const void* c, const void* Q, const void* R, const void* M, const void* q, const void* r,
                    const void* x0, void* x, void* u, void* lam, int32_t* status, void* workspace,
                    size_t workspace_bytes, const lqr_opts* opts) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.method != LQR_METHOD_SCAN) return fail(LQR_EINVAL, "lqr_kkt_resolve reuses the factors of the scan method");
    if (o.warm_x || o.warm_u || o.warm_lam) return fail(LQR_EINVAL, "lqr_kkt_resolve takes no warm start");
    o.method = kResolve;
    return solve_impl(h, stream, batch, N, n, m, A, B, c, Q, R, M, q, r, x0, x, u, lam, status, workspace,
                      workspace_bytes, o, h->find(batch, N, n, m, o.dtype));
}

size_t lqr_noalloc_workspace_bytes(void) { return kNoAllocBytes; }

}  // extern "C"

namespace {
// element counts of one instance's arrays, in ABI field order
void field_elems(int N, int n, int m, int64_t (&in)[9], int64_t (&out)[3]) {
    const int64_t nn = (int64_t)n * n;
    in[0] = N * nn;                  // A
    in[1] = (int64_t)N * n * m;      // B
    in[2] = (int64_t)N * n;          // c
    in[3] = (int64_t)(N + 1) * nn;   // Q
    in[4] = (int64_t)N * m * m;      // R
    in[5] = (int64_t)N * n * m;      // M
    in[6] = (int64_t)(N + 1) * n;    // q
    in[7] = (int64_t)N * m;          // r
    in[8] = n;                       // x0
    out[0] = (int64_t)(N + 1) * n;   // x
    out[1] = (int64_t)N * m;         // u
    out[2] = (int64_t)(N + 1) * n;   // lam
}

struct RaggedGroup {
    int N, n, m;
    std::vector<int> ids;
};

int ragged_groups(int64_t count, const lqr_problem* probs, size_t es, std::vector<RaggedGroup>& groups) {
    if (count < 1) return fail(LQR_EINVAL, "count must be >= 1");
    if (!probs) return fail(LQR_EINVAL, "null problem table");
    std::map<std::tuple<int, int, int>, size_t> where;
    for (int64_t i = 0; i < count; ++i) {
        const lqr_problem& p = probs[i];
        LCHK(check_dims(1, p.N, p.n, p.m));
        const void* ptrs[] = {p.A, p.B, p.c, p.Q, p.R, p.M, p.q, p.r, p.x0, p.x, p.u, p.lam};
        for (const void* q : ptrs) {
            if (!q) return fail(LQR_EINVAL, "problem %lld has a null array", (long long)i);
            if (!aligned(q, es)) return fail(LQR_EINVAL, "problem %lld has a misaligned array", (long long)i);
        }
        const auto key = std::make_tuple(p.N, p.n, p.m);
        auto it = where.find(key);
        if (it == where.end()) {
            where[key] = groups.size();
            groups.push_back(RaggedGroup{p.N, p.n, p.m, {}});
            it = where.find(key);
        }
        groups[it->second].ids.push_back((int)i);
    }
    return LQR_OK;
}

// bytes of one group's packed arrays + its solve workspace
struct GroupBytes {
    size_t in, out, st, rel, solve, total;
};
GroupBytes group_bytes(const lqr_handle_s* h, const RaggedGroup& g, size_t es, const lqr_opts& o) {
    int64_t ie[9], oe[3];
    field_elems(g.N, g.n, g.m, ie, oe);
    int64_t in = 0, out = 0;
    for (int64_t v : ie) in += v;
    for (int64_t v : oe) out += v;
    const int64_t k = (int64_t)g.ids.size();
    GroupBytes b;
    b.in = (size_t)align_up(k * in * (int64_t)es, 256);
    b.out = (size_t)align_up(k * out * (int64_t)es, 256);
    b.st = (size_t)align_up(k * 4, 256);
    b.rel = (size_t)align_up(k * 8, 256);
    const Tuning* tun = h ? h->find(k, g.N, g.n, g.m, o.dtype) : nullptr;
    b.solve = solve_bytes(k, g.N, g.n, g.m, es, o, tun);
    b.total = b.in + b.out + b.st + b.rel + b.solve;
    return b;
}

int pack_launch(hipStream_t s, bool gather, const std::vector<void*>& ptrs, const std::vector<int>& ids,
                char* packed, int64_t elems, size_t es) {
    const int64_t words = elems * (int64_t)es / 4;
    for (size_t c0 = 0; c0 < ptrs.size(); c0 += kPackTable) {
        PackTable t;
        std::memset(&t, 0, sizeof t);
        t.count = (int)std::min<size_t>(kPackTable, ptrs.size() - c0);
        for (int j = 0; j < t.count; ++j) {
            t.p[j] = ptrs[c0 + j];
            t.idx[j] = ids[c0 + j];
        }
        const int64_t gx = std::min<int64_t>((words + 255) / 256, 64);
        uint32_t* pk = reinterpret_cast<uint32_t*>(packed + c0 * elems * es);
        Timer* tm = current_timer();
        if (tm) tm->before(s, F_PACK, 0, 2.0 * words * 4 * t.count, 0);
        if (gather)
            hipLaunchKernelGGL(k_pack<true>, dim3((unsigned)gx, (unsigned)t.count), dim3(256), 0, s, t, pk, words);
        else
            hipLaunchKernelGGL(k_pack<false>, dim3((unsigned)gx, (unsigned)t.count), dim3(256), 0, s, t, pk, words);
        if (tm) tm->after(s);
        HIPCHK(hipGetLastError());
    }
    return LQR_OK;
}
}  // namespace

extern "C" {

int lqr_ragged_workspace_size(lqr_handle_t h, int64_t count, const lqr_problem* probs, const lqr_opts* opts,
                              size_t* bytes) {
    if (!bytes) return fail(LQR_EINVAL, "null output pointer");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    std::vector<RaggedGroup> groups;
    LCHK(ragged_groups(count, probs, es, groups));
    size_t most = 0;
    for (const auto& g : groups) most = std::max(most, group_bytes(h, g, es, o).total);
    *bytes = most;
    return LQR_OK;
}

int lqr_kkt_solve_ragged(lqr_handle_t h, void* stream, int64_t count, const lqr_problem* probs, int32_t* status,
                         void* workspace, size_t workspace_bytes, const lqr_opts* opts) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    if (o.warm_x || o.warm_u || o.warm_lam) return fail(LQR_EINVAL, "warm starts are per batch, not per ragged call");
    if (!status || !workspace) return fail(LQR_EINVAL, "null status or workspace");
    if (!aligned(status, 4) || !aligned(workspace, 256)) return fail(LQR_EINVAL, "misaligned status or workspace");
    if (count > 0x7fffffff) return fail(LQR_EINVAL, "count too large");
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    std::vector<RaggedGroup> groups;
    LCHK(ragged_groups(count, probs, es, groups));
    for (const auto& g : groups)
        if (group_bytes(h, g, es, o).total > workspace_bytes)
            return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu a group needs", workspace_bytes,
                        group_bytes(h, g, es, o).total);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    double* rel_out = o.resid_out;
    TimerScope ts_scope(h->timing ? &h->timer : nullptr);
    for (const auto& g : groups) {
        const GroupBytes gb = group_bytes(h, g, es, o);
        const int64_t k = (int64_t)g.ids.size();
        char* base = static_cast<char*>(workspace);
        char* pin = base;
        char* pout = pin + gb.in;
        int32_t* pst = reinterpret_cast<int32_t*>(pout + gb.out);
        double* prel = reinterpret_cast<double*>(reinterpret_cast<char*>(pst) + gb.st);
        char* pws = reinterpret_cast<char*>(prel) + gb.rel;
        int64_t ie[9], oe[3];
        field_elems(g.N, g.n, g.m, ie, oe);
        // gather the inputs field by field into batch-major arrays
        const void* fin[9];
        char* cur = pin;
        for (int f = 0; f < 9; ++f) {
            std::vector<void*> ptrs;
            for (int id : g.ids) {
                const lqr_problem& p = probs[id];
                const void* a[] = {p.A, p.B, p.c, p.Q, p.R, p.M, p.q, p.r, p.x0};
                ptrs.push_back(const_cast<void*>(a[f]));
            }
            LCHK(pack_launch(s, true, ptrs, g.ids, cur, ie[f], es));
            fin[f] = cur;
            cur += k * ie[f] * (int64_t)es;
        }
        void* fout[3];
        cur = pout;
        for (int f = 0; f < 3; ++f) {
            fout[f] = cur;
            cur += k * oe[f] * (int64_t)es;
        }
        lqr_opts og = o;
        og.resid_out = rel_out ? prel : nullptr;
        og.sync_status = 0;
        LCHK(solve_impl(h, stream, k, g.N, g.n, g.m, fin[0], fin[1], fin[2], fin[3], fin[4], fin[5], fin[6],
                        fin[7], fin[8], fout[0], fout[1], fout[2], pst, pws, gb.solve, og,
                        h->find(k, g.N, g.n, g.m, o.dtype)));
        // scatter the solutions and the status words back
        for (int f = 0; f < 3; ++f) {
            std::vector<void*> ptrs;
            for (int id : g.ids) {
                const lqr_problem& p = probs[id];
                void* a[] = {p.x, p.u, p.lam};
                ptrs.push_back(a[f]);
            }
            LCHK(pack_launch(s, false, ptrs, g.ids, static_cast<char*>(fout[f]), oe[f], es));
        }
        for (size_t c0 = 0; c0 < g.ids.size(); c0 += kPackTable) {
            PackTable t;
            std::memset(&t, 0, sizeof t);
            t.count = (int)std::min<size_t>(kPackTable, g.ids.size() - c0);
            for (int j = 0; j < t.count; ++j) t.idx[j] = g.ids[c0 + j];
            hipLaunchKernelGGL(k_unpack_status<double>, dim3(1), dim3(64), 0, s, t, pst + c0, prel + c0, status, rel_out);
            HIPCHK(hipGetLastError());
        }
    }
    if (o.sync_status) return sync_status_check(s, status, count);
    return LQR_OK;
}

}  // extern "C"

namespace {
Tuning from_abi(const lqr_tuning& t) {
    Tuning tu;
    tu.engine = t.engine;
    tu.fused = t.fused;
    tu.big_grid = t.big_grid;
    tu.split = t.split;
    tu.chunk = t.chunk;
    tu.sweep = t.sweep;
    tu.fwd_seq = t.fwd_seq;
    tu.streams = t.streams;
    return tu;
}
void to_abi(const Tuning& t, float ms, lqr_tuning* o) {
    o->engine = t.engine;
    o->fused = t.fused;
    o->big_grid = t.big_grid;
    o->ms = ms;
    o->split = t.split;
    o->chunk = t.chunk;
    o->sweep = t.sweep;
    o->fwd_seq = t.fwd_seq;
    o->streams = t.streams;
}

int check_tuning(int N, int n, int m, const Tuning& t) {
    if (t.engine < 0 || t.engine > 2 || t.fused < -1 || t.fused > 2 || t.big_grid < 0 || t.split < 0 || t.split > 2 ||
        t.chunk < 0 || t.sweep < 0 || t.fwd_seq < 0 || t.fwd_seq > 1 || t.streams < 0 || t.streams > kMaxParts)
        return fail(LQR_EINVAL,
                    "bad tuning (engine %d, fused %d, big_grid %d, split %d, chunk %d, sweep %d, fwd_seq %d, streams %d)",
                    t.engine, t.fused, t.big_grid, t.split, t.chunk, t.sweep, t.fwd_seq, t.streams);
    const bool big = t.engine == 2 || pick_ts(n, m) == kBigTS;
    if (t.split && (big || t.fused == 2))
        return fail(LQR_EINVAL, "the split and chunked schedules run on the wavefront engine with level-by-level launches");
    if (t.split == 2 && (t.chunk < 1 || t.sweep < 1 || t.sweep > N + 1))
        return fail(LQR_EINVAL, "chunked schedule needs chunk >= 1 and 1 <= sweep <= N+1 (chunk %d, sweep %d)", t.chunk,
                    t.sweep);
    if (t.engine == 1 && pick_ts(n, m) == kBigTS)
        return fail(LQR_EINVAL, "the wavefront engine takes orders up to 64 (n=%d m=%d)", n, m);
    if (t.fused == 2 && big)
        return fail(LQR_EINVAL, "the one-launch solve runs on the wavefront engine (orders up to 64)");
    if (t.fwd_seq && t.fused == 2)
        return fail(LQR_EINVAL, "the one-launch solve has its own vector passes (fwd_seq needs fused 0 or 1)");
    lqr_opts o;
    lqr_opts_default(&o, LQR_F32);
    if (!sched_fits(make_plan(1, N, n, m, 4, o, &t)))
        return fail(LQR_EINVAL, "chunked schedule does not fit the tree records of N=%d", N);
    return LQR_OK;
}

// bucket of a size for the tuning cache: the next power of two
int64_t bucket(int64_t v) {
    int64_t b = 1;
    while (b < v) b <<= 1;
    return b;
}
}  // namespace

const Tuning* lqr_handle_s::find(int64_t batch, int N, int n, int m, int dtype) const {
    auto it = tuned.find(std::make_tuple(batch, N, n, m, dtype));
    if (it != tuned.end()) return &it->second;
    auto jt = cached.find(std::make_tuple(bucket(batch), (int)bucket(N), n, m, dtype));
    if (jt != cached.end()) return &jt->second;
    return nullptr;
}

extern "C" {

static_assert(sizeof(lqr_problem_desc) == sizeof(RaggedDesc), "descriptor layout");
static_assert(offsetof(lqr_problem_desc, in_off) == offsetof(RaggedDesc, in_off), "descriptor layout");
static_assert(offsetof(lqr_problem_desc, out_off) == offsetof(RaggedDesc, out_off), "descriptor layout");

}  // extern "C"

namespace {
// workspace of a device-descriptor ragged call: work counters | slots of
// records | FP64 partial sums per slot | FP64 redo slots
struct DevRaggedLayout {
    int64_t slot_elems, dslot, slot64, redo_slots;
    size_t cnt_off, rec_off, dbl_off, redo_off, total;
};

int dev_ragged_layout(int64_t count, int slots, int maxN, int maxd, const lqr_opts& o, DevRaggedLayout& l) {
    if (count < 1 || count > 0x7fffffff) return fail(LQR_EINVAL, "count must be in 1..2^31-1");
    if (slots < 1 || slots > 65536) return fail(LQR_EINVAL, "slots must be in 1..65536 (got %d)", slots);
    if (maxN < 1 || maxN + 1 > (1 << (LQR_MAXLEV - 2))) return fail(LQR_EINVAL, "bad maxN %d", maxN);
    if (maxd < 1 || maxd > 64) return fail(LQR_EINVAL, "maxd must be in 1..64 (the wavefront classes; got %d)", maxd);
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    Plan p;
    std::memset(&p, 0, sizeof p);
    plan_records(p, maxN, maxd, maxd, false);
    l.slot_elems = p.stride;
    l.dslot = align_up(p.dstride + 1, 8);
    Plan r = p;
    redo_records(r);
    l.slot64 = r.stride;
    l.redo_slots = (o.dtype == LQR_F32 && o.fallback) ? std::min<int64_t>(slots, kRedoSlots) : 0;
    l.cnt_off = 0;
    l.rec_off = 256;
    l.dbl_off = l.rec_off + (size_t)align_up((int64_t)slots * l.slot_elems * (int64_t)es, 256);
    l.redo_off = l.dbl_off + (size_t)align_up((int64_t)slots * l.dslot * 8, 256);
    l.total = l.redo_off + (size_t)align_up(l.redo_slots * l.slot64 * 8, 256);
    return LQR_OK;
}

template <typename S>
int solve_ragged_dev(hipStream_t s, int64_t count, const lqr_problem_desc* descs, const void* in, void* out,
                     int32_t* status, int slots, int maxN, int maxd, char* ws, const DevRaggedLayout& l,
                     const lqr_opts& o) {
    RaggedArgs<S> a;
    std::memset(&a, 0, sizeof a);
    a.desc = reinterpret_cast<const RaggedDesc*>(descs);
    a.count = count;
    a.in = (const S*)in;
    a.out = (S*)out;
    a.status = status;
    a.rel = o.resid_out;
    a.ws = (S*)(ws + l.rec_off);
    a.slot_elems = l.slot_elems;
    a.dws = (double*)(ws + l.dbl_off);
    a.dslot = l.dslot;
    a.ws64 = (double*)(ws + l.redo_off);
    a.slot64 = l.slot64;
    a.warm_x = (const S*)o.warm_x;
    a.warm_u = (const S*)o.warm_u;
    a.warm_lam = (const S*)o.warm_lam;
    a.maxN = maxN;
    a.maxd = maxd;
    a.refine = o.refine_sweeps;
    a.fallback = sizeof(S) == 4 ? o.fallback : 0;
    a.cond_thr = o.cond_threshold;
    a.refine_tol = o.refine_tol;
    int32_t* counters = (int32_t*)(ws + l.cnt_off);
    LCHK(launch_nt(256, F_CLEAR, 0, 0, k_clear<int32_t>, 1, s, counters, (int64_t)64));
    LCHK(launch_nt(256, F_CLEAR, 0, 0, k_ragged_check<S>, (count + 255) / 256, s, a));
    const int rs = (int)l.redo_slots;
    const int classes[] = {1, 2, 3, 4, 5, 6, 8};
    for (int ci = 0; ci < 7; ++ci) {
        int32_t* c = counters + 2 * ci;
        int rc;
        switch (classes[ci]) {
            case 1: rc = run_ragged<S, 1>(s, a, slots, rs, c); break;
            case 2: rc = run_ragged<S, 2>(s, a, slots, rs, c); break;
            case 3: rc = run_ragged<S, 3>(s, a, slots, rs, c); break;
            case 4: rc = run_ragged<S, 4>(s, a, slots, rs, c); break;
            case 5: rc = run_ragged<S, 5>(s, a, slots, rs, c); break;
            case 6: rc = run_ragged<S, 6>(s, a, slots, rs, c); break;
            default: rc = run_ragged<S, 8>(s, a, slots, rs, c); break;
        }
        LCHK(rc);
    }
    return LQR_OK;
}
}  // namespace

extern "C" {

int lqr_ragged_dev_workspace_size(int64_t count, int32_t slots, int32_t maxN, int32_t maxd, const lqr_opts* opts,
                                  size_t* bytes) {
    if (!bytes) return fail(LQR_EINVAL, "null output pointer");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    DevRaggedLayout l;
    LCHK(dev_ragged_layout(count, slots, maxN, maxd, o, l));
    *bytes = l.total;
    return LQR_OK;
}

int lqr_kkt_solve_ragged_dev(lqr_handle_t h, void* stream, int64_t count, const lqr_problem_desc* descs,
                             const void* in, void* out, int32_t* status, int32_t slots, int32_t maxN, int32_t maxd,
                             void* workspace, size_t workspace_bytes, const lqr_opts* opts) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    if (o.method != LQR_METHOD_SCAN) return fail(LQR_EINVAL, "the ragged persistent solve is the scan method");
    if (o.refine_sweeps < 0 || o.refine_sweeps > 4) return fail(LQR_EINVAL, "refine_sweeps must be in 0..4");
    if (!(o.refine_tol > 0.0) || !(o.cond_threshold > 1.0)) return fail(LQR_EINVAL, "bad refine_tol / cond_threshold");
    DevRaggedLayout l;
    LCHK(dev_ragged_layout(count, slots, maxN, maxd, o, l));
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    if (!descs || !in || !out || !status || !workspace) return fail(LQR_EINVAL, "null pointer argument");
    if (!aligned(descs, 8) || !aligned(in, es) || !aligned(out, es) || !aligned(status, 4) || !aligned(workspace, 256))
        return fail(LQR_EINVAL, "misaligned argument");
    if (o.resid_out && !aligned(o.resid_out, 8)) return fail(LQR_EINVAL, "misaligned resid_out");
    const bool has_warm = o.warm_x || o.warm_u || o.warm_lam;
    if (has_warm && (!o.warm_x || !o.warm_u || !o.warm_lam)) return fail(LQR_EINVAL, "warm start needs x, u and lam");
    if (workspace_bytes < l.total)
        return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, l.total);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    int rc;
    {
        TimerScope ts_scope(h->timing ? &h->timer : nullptr);
        rc = o.dtype == LQR_F32 ? solve_ragged_dev<float>(s, count, descs, in, out, status, slots, maxN, maxd,
                                                          (char*)workspace, l, o)
                                : solve_ragged_dev<double>(s, count, descs, in, out, status, slots, maxN, maxd,
                                                           (char*)workspace, l, o);
    }
    if (rc != LQR_OK || !o.sync_status) return rc;
    return sync_status_check(s, status, count);
}

int lqr_set_tuning(lqr_handle_t h, int64_t batch, int N, int n, int m, int32_t dtype, const lqr_tuning* t) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    LCHK(check_dims(batch, N, n, m));
    const auto key = std::make_tuple(batch, N, n, m, (int)dtype);
    if (!t) {
        h->tuned.erase(key);
        h->cached.erase(std::make_tuple(bucket(batch), (int)bucket(N), n, m, (int)dtype));
        return LQR_OK;
    }
    const Tuning tu = from_abi(*t);
    LCHK(check_tuning(N, n, m, tu));
    h->tuned[key] = tu;
    return LQR_OK;
}

int lqr_autotune(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, const void* A, const void* B,
                 const void* c, const void* Q, const void* R, const void* M, const void* q, const void* r,
                 const void* x0, void* x, void* u, void* lam, int32_t* status, void* workspace,
                 size_t workspace_bytes, const lqr_opts* opts, int reps, lqr_tuning* best) {
    if (!h || !best) return fail(LQR_EINVAL, "null handle or result");
    if (reps < 1 || reps > 100) return fail(LQR_EINVAL, "reps must be in 1..100");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    o.sync_status = 0;
    LCHK(check_dims(batch, N, n, m));
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    // candidate mappings: engine x schedule of the reverse scan x form of the
    // vector passes (x matrix-core grid)
    std::vector<Tuning> cands;
    const bool small_ok = pick_ts(n, m) != kBigTS;
    if (small_ok) {
        for (int fs : {0, 1}) {
            for (int fu : {0, 1}) {
                if (fs && fu) continue;   // the sequential passes are already per instance
                Tuning t; t.engine = 1; t.fused = fu; t.fwd_seq = fs; cands.push_back(t);
            }
            Tuning sp; sp.engine = 1; sp.fused = 0; sp.fwd_seq = fs; sp.split = 1; cands.push_back(sp);
            for (int ch : {1, 4, 8, 16, 32}) {
                if (ch > 1 && ch >= N) continue;
                Tuning t; t.engine = 1; t.fused = 0; t.fwd_seq = fs; t.split = 2; t.chunk = ch; t.sweep = 1;
                cands.push_back(t);
            }
        }
        Tuning one; one.engine = 1; one.fused = 2; cands.push_back(one);
    }
    for (int fs : {0, 1})
        for (int fu : {0, 1}) {
            if (fs && fu) continue;
            for (int g : {256, 512, 1024}) {
                Tuning t; t.engine = 2; t.fused = fu; t.fwd_seq = fs; t.big_grid = g; cands.push_back(t);
            }
        }
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<int32_t> st((size_t)batch);
    float best_ms = -1.0f;
    Tuning best_t;
    // time one candidate: *ms < 0 if it does not fit or its status is not clean
    auto time_one = [&](const Tuning& t, float* ms) -> int {
        *ms = -1.f;
        const Plan pl = make_plan(batch, N, n, m, es, o, &t);
        if (!sched_fits(pl) || solve_bytes(batch, N, n, m, es, o, &t) > workspace_bytes) return LQR_OK;
        auto run = [&]() {
            return solve_impl(h, stream, batch, N, n, m, A, B, c, Q, R, M, q, r, x0, x, u, lam, status, workspace,
                              workspace_bytes, o, &t);
        };
        LCHK(run());   // warm-up (and the status check below)
        if (hipMemcpyAsync(st.data(), status, sizeof(int32_t) * (size_t)batch, hipMemcpyDeviceToHost, s) !=
                hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return fail(LQR_EDEVICE, "reading the status words failed");
        bool clean = true;
        for (int32_t v : st) clean = clean && (v & ~LQR_ST_FP64_FALLBACK) == 0;
        if (!clean) return LQR_OK;
        (void)hipEventRecord(e0, s);
        for (int i = 0; i < reps; ++i) LCHK(run());
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return fail(LQR_EDEVICE, "timing event failed");
        float t_ms = 0.f;
        (void)hipEventElapsedTime(&t_ms, e0, e1);
        *ms = t_ms / (float)reps;
        if (best_ms < 0.f || *ms < best_ms) {
            best_ms = *ms;
            best_t = t;
        }
        return LQR_OK;
    };
    int rc = LQR_OK;
    std::vector<std::pair<float, Tuning>> timed;
    for (const Tuning& t : cands) {
        float ms;
        if ((rc = time_one(t, &ms)) != LQR_OK) break;
        if (ms >= 0.f) timed.emplace_back(ms, t);
    }
    // the three fastest mappings again with the batch split over 2 and 4
    // streams (parts of at least 2 instances)
    std::stable_sort(timed.begin(), timed.end(),
                     [](const std::pair<float, Tuning>& x1, const std::pair<float, Tuning>& x2) {
                         return x1.first < x2.first;
                     });
    for (size_t i = 0; i < timed.size() && i < 3 && rc == LQR_OK; ++i)
        for (int k : {2, 4}) {
            if (batch < 2 * k) continue;
            Tuning t = timed[i].second;
            t.streams = k;
            float ms;
            if ((rc = time_one(t, &ms)) != LQR_OK) break;
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LQR_OK) return rc;
    if (best_ms < 0.f) return fail(LQR_ENOMEM, "no candidate mapping fits the workspace with a clean status");
    h->tuned[std::make_tuple(batch, N, n, m, (int)o.dtype)] = best_t;
    h->cached[std::make_tuple(bucket(batch), (int)bucket(N), n, m, (int)o.dtype)] = best_t;
    to_abi(best_t, best_ms, best);
    return LQR_OK;
}

// Tuning cache file: one line per shape bucket,
//   "lqr-tune-1 <arch> <dtype> <n> <m> <N bucket> <batch bucket> <engine> <fused> <big_grid> <split> <chunk>
//    <sweep> <fwd_seq> [<streams>]"
// (sizes rounded up to powers of two; a line without the last field maps
// to one stream).  Lines of another device architecture are kept in the
// file but not loaded.
int lqr_tuning_save(lqr_handle_t h, const char* path) {
    if (!h || !path) return fail(LQR_EINVAL, "null handle or path");
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, h->device));
    const std::string arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    std::vector<std::string> keep;
    if (FILE* f = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof line, f)) {
            char a[64] = {0};
            if (std::sscanf(line, "lqr-tune-1 %63s", a) == 1 && arch != a) keep.push_back(line);
        }
        std::fclose(f);
    }
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(LQR_EINVAL, "cannot write %s", tmp.c_str());
    for (const auto& l : keep) std::fputs(l.c_str(), f);
    for (const auto& kv : h->cached) {
        const auto& k = kv.first;
        const Tuning& t = kv.second;
        std::fprintf(f, "lqr-tune-1 %s %d %d %d %lld %lld %d %d %d %d %d %d %d %d\n", arch.c_str(), std::get<4>(k),
                     std::get<2>(k), std::get<3>(k), (long long)std::get<1>(k), (long long)std::get<0>(k), t.engine,
                     t.fused, t.big_grid, t.split, t.chunk, t.sweep, t.fwd_seq, t.streams);
    }
    std::fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) return fail(LQR_EINVAL, "cannot replace %s", path);
    return LQR_OK;
}

int lqr_tuning_load(lqr_handle_t h, const char* path) {
    if (!h || !path) return fail(LQR_EINVAL, "null handle or path");
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, h->device));
    const std::string arch = std::string(prop.gcnArchName).substr(0, std::string(prop.gcnArchName).find(':'));
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(LQR_EINVAL, "cannot read %s", path);
    char line[512];
    int loaded = 0;
    while (std::fgets(line, sizeof line, f)) {
        char a[64] = {0};
        int dt, n, m;
        long long Nb, Bb;
        Tuning t;
        const int got = std::sscanf(line, "lqr-tune-1 %63s %d %d %d %lld %lld %d %d %d %d %d %d %d %d", a, &dt, &n, &m,
                                    &Nb, &Bb, &t.engine, &t.fused, &t.big_grid, &t.split, &t.chunk, &t.sweep,
                                    &t.fwd_seq, &t.streams);
        if (got != 13 && got != 14) continue;
        if (arch != a || n < 1 || m < 1 || Nb < 1 || Bb < 1) continue;
        if (check_tuning((int)Nb, n, m, t) != LQR_OK) continue;
        h->cached[std::make_tuple((int64_t)Bb, (int)Nb, n, m, dt)] = t;
        ++loaded;
    }
    std::fclose(f);
    return loaded;
}

int lqr_autotune_workspace_size(int64_t batch, int N, int n, int m, const lqr_opts* opts, size_t* bytes) {
    if (!bytes) return fail(LQR_EINVAL, "null output pointer");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    LCHK(check_dims(batch, N, n, m));
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    // the largest of: each engine, on one stream and split over 2 and 4
    size_t need = 0;
    for (int k : {0, 2, 4}) {
        Tuning t;
        t.engine = 2;
        t.big_grid = 1024;
        t.streams = k;
        need = std::max(need, solve_bytes(batch, N, n, m, es, o, &t));
        if (pick_ts(n, m) != kBigTS) {
            Tuning w;
            w.engine = 1;
            w.streams = k;
            need = std::max(need, solve_bytes(batch, N, n, m, es, o, &w));
        }
    }
    *bytes = need;
    return LQR_OK;
}

int lqr_kkt_residual(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, int32_t dtype,
                     const void* A, const void* B, const void* c, const void* Q, const void* R, const void* M,
                     const void* q, const void* r, const void* x0, const void* x, const void* u,
                     const void* lam, double* rel, void* workspace, size_t workspace_bytes) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    LCHK(check_dims(batch, N, n, m));
    if (dtype != LQR_F32 && dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", dtype);
    const void* ptrs[] = {A, B, c, Q, R, M, q, r, x0, x, u, lam, rel, workspace};
    for (const void* ptr : ptrs)
        if (!ptr) return fail(LQR_EINVAL, "null pointer argument");
    lqr_opts o;
    lqr_opts_default(&o, dtype);
    const size_t es = dtype == LQR_F32 ? 4 : 8;
    const Tuning* tun = h->find(batch, N, n, m, dtype);
    Plan p = make_plan(batch, N, n, m, es, o, tun);
    const Layout lay = layout(p, es);
    if (workspace_bytes < lay.total)
        return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, lay.total);
    p.o_scr = (int64_t)lay.scr_off;
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    char* wsb = (char*)workspace;
    double* dws = (double*)(wsb + lay.dbl_off);
    const int ts = pick_ts(n, m, tun);
    TimerScope ts_scope(h->timing ? &h->timer : nullptr);
    if (dtype == LQR_F32) {
        In<float> in{(const float*)A, (const float*)B, (const float*)c, (const float*)Q, (const float*)R,
                     (const float*)M, (const float*)q, (const float*)r, (const float*)x0};
        return dispatch_resid<float>(ts, p, s, in, (const float*)x, (const float*)u, (const float*)lam,
                                     (float*)wsb, dws, rel);
    }
    In<double> in{(const double*)A, (const double*)B, (const double*)c, (const double*)Q, (const double*)R,
                  (const double*)M, (const double*)q, (const double*)r, (const double*)x0};
    return dispatch_resid<double>(ts, p, s, in, (const double*)x, (const double*)u, (const double*)lam,
                                  (double*)wsb, dws, rel);
}

int lqr_kkt_factors(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, int32_t dtype,
                    const void* workspace, size_t workspace_bytes, void* P, void* p, void* K, void* kff) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    LCHK(check_dims(batch, N, n, m));
    if (dtype != LQR_F32 && dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", dtype);
    if (!workspace || !P || !p || !K || !kff) return fail(LQR_EINVAL, "null pointer argument");
    lqr_opts o;
    lqr_opts_default(&o, dtype);
    const size_t es = dtype == LQR_F32 ? 4 : 8;
    const void* outs[] = {P, p, K, kff};
    for (const void* ptr : outs)
        if (!aligned(ptr, es)) return fail(LQR_EINVAL, "misaligned output");
    const Tuning* tun = h->find(batch, N, n, m, dtype);
    const size_t need = solve_bytes(batch, N, n, m, es, o, tun);
    if (workspace_bytes < need)
        return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu of this shape", workspace_bytes, need);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    // the records of each part of a batch split over streams sit in its slice
    const Parts pt = parts_of(batch, N, n, m, es, o, tun);
    for (int j = 0; j < pt.count; ++j) {
        const int64_t b0 = j * pt.size, cnt = std::min(pt.size, batch - b0);
        const Plan pl = make_plan(cnt, N, n, m, es, o, tun);
        const char* wsb = (const char*)workspace + (pt.count > 1 ? (size_t)j * pt.bytes : 0);
        const int64_t grid = cnt * (N + 1), sN1 = b0 * (N + 1), sN = b0 * N;
        if (dtype == LQR_F32)
            hipLaunchKernelGGL(k_factors<float>, dim3((unsigned)grid), dim3(256), 0, s, pl, (const float*)wsb,
                               (float*)P + sN1 * n * n, (float*)p + sN1 * n, (float*)K + sN * m * n,
                               (float*)kff + sN * m);
        else
            hipLaunchKernelGGL(k_factors<double>, dim3((unsigned)grid), dim3(256), 0, s, pl, (const double*)wsb,
                               (double*)P + sN1 * n * n, (double*)p + sN1 * n, (double*)K + sN * m * n,
                               (double*)kff + sN * m);
        HIPCHK(hipGetLastError());
    }
    return LQR_OK;
}

int lqr_qp_build(lqr_handle_t h, void* stream, int64_t batch, int N, int n, int m, int p, int nc, int32_t dtype,
                 const void* Ex, const void* Eu, const void* e, const void* W, const void* Gx, const void* Gu,
                 const void* g, const void* mu, const void* delta, void* Q, void* M, void* R, void* q, void* r) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    if (batch < 1 || N < 1 || n < 1 || m < 1 || p < 1 || nc < 0)
        return fail(LQR_EINVAL, "bad sizes (batch %lld, N %d, n %d, m %d, p %d, nc %d)", (long long)batch, N, n, m, p,
                    nc);
    if (dtype != LQR_F32 && dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", dtype);
    const size_t es = dtype == LQR_F32 ? 4 : 8;
    const size_t lds = es * ((size_t)p * (n + m) + p + 2 * (size_t)nc);
    if (lds > 65536) return fail(LQR_EINVAL, "p (n + m) too large for one workgroup's LDS (%zu bytes)", lds);
    if (batch * (int64_t)(N + 1) > 0x7fffffff) return fail(LQR_EINVAL, "batch*(N+1) exceeds the grid limit");
    const void* need[] = {Ex, Eu, e, W, Q, M, R, q, r};
    for (const void* ptr : need)
        if (!ptr || !aligned(ptr, es)) return fail(LQR_EINVAL, "null or misaligned array");
    if (nc > 0) {
        const void* cons[] = {Gx, Gu, g, mu, delta};
        for (const void* ptr : cons)
            if (!ptr || !aligned(ptr, es)) return fail(LQR_EINVAL, "null or misaligned constraint array");
    }
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)(batch * (N + 1)));
    if (dtype == LQR_F32) {
        QpArgs<float> a{batch, N, n, m, p, nc, (const float*)Ex, (const float*)Eu, (const float*)e, (const float*)W,
                        (const float*)Gx, (const float*)Gu, (const float*)g, (const float*)mu,
                        (const float*)delta, (float*)Q, (float*)M, (float*)R, (float*)q, (float*)r};
        hipLaunchKernelGGL(k_qp_build<float>, grid, dim3(256), lds, s, a);
    } else {
        QpArgs<double> a{batch, N, n, m, p, nc, (const double*)Ex, (const double*)Eu, (const double*)e,
                         (const double*)W, (const double*)Gx, (const double*)Gu, (const double*)g,
                         (const double*)mu, (const double*)delta, (double*)Q, (double*)M, (double*)R, (double*)q,
                         (double*)r};
        hipLaunchKernelGGL(k_qp_build<double>, grid, dim3(256), lds, s, a);
    }
    HIPCHK(hipGetLastError());
    return LQR_OK;
}

}  // extern "C"

namespace {
// workspace of lqr_sqp_solve: the subproblem's arrays, its solution, the
// line search's sums, then the KKT solve's own workspace
struct SqpLayout {
    size_t off[22];
    size_t solve_off, total;
};

SqpLayout sqp_layout(lqr_handle_t h, int64_t B, int N, int n, int m, int nc, const lqr_opts& o) {
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    const int64_t p = n + m, N1 = N + 1;
    const int64_t elems[22] = {B * N * n * n, B * N * n * m, B * N * n, B * n,            // A B c x0
                               B * N1 * p * n, B * N * p * m, B * N1 * p, B * N1 * p * p,  // Ex Eu e W
                               B * N1 * nc * n, B * N * nc * m, B * N1 * nc,               // Gx Gu g
                               B * N1 * n * n, B * N * n * m, B * N * m * m, B * N1 * n, B * N * m,   // Q M R q r
                               B * N1 * n, B * N * m, B * N1 * n,                           // dx du lqp
                               B * (kAlphas + 1), B * (kAlphas + 1), B};                     // th J dJ (double)
    SqpLayout l;
    size_t cur = 0;
    for (int i = 0; i < 22; ++i) {
        l.off[i] = cur;
        cur += (size_t)align_up(elems[i] * (int64_t)(i >= 19 ? 8 : es), 256);
    }
    l.solve_off = cur;
    const Tuning* tun = h ? h->find(B, N, n, m, o.dtype) : nullptr;
    l.total = cur + solve_bytes(B, N, n, m, es, o, tun);
    return l;
}

int sqp_check(int64_t batch, int N, int n, int m, int nc, const lqr_opts& o) {
    LCHK(check_dims(batch, N, n, m));
    if (n > 64 || m > 64 || nc < 0 || nc > 64)
        return fail(LQR_EINVAL, "the SQP kernels take n, m, nc <= 64 (n %d m %d nc %d)", n, m, nc);
    if (o.dtype != LQR_F32 && o.dtype != LQR_F64) return fail(LQR_EINVAL, "bad dtype %d", o.dtype);
    if (o.method != LQR_METHOD_SCAN) return fail(LQR_EINVAL, "the SQP iteration uses the scan method");
    if (o.warm_x || o.warm_u || o.warm_lam) return fail(LQR_EINVAL, "the SQP iteration takes no warm start");
    return LQR_OK;
}

template <typename S>
int sqp_run(lqr_handle_t h, hipStream_t s, const lqr_bilinear_model& mdl, int iters, double theta_max, S* X, S* U,
            S* L, S* alpha_out, int32_t* status, char* ws, size_t ws_bytes, const SqpLayout& l, const lqr_opts& o) {
    SqpModel<S> md;
    md.batch = mdl.batch; md.N = mdl.N; md.n = mdl.n; md.m = mdl.m; md.nc = mdl.nc;
    md.A = (const S*)mdl.A; md.B = (const S*)mdl.B; md.c = (const S*)mdl.c; md.P = (const S*)mdl.P;
    md.V = (const S*)mdl.V; md.xr = (const S*)mdl.xr; md.ur = (const S*)mdl.ur; md.wx = (const S*)mdl.wx;
    md.wu = (const S*)mdl.wu; md.Gx = (const S*)mdl.Gx; md.Gu = (const S*)mdl.Gu; md.g0 = (const S*)mdl.g0;
    md.mu = (const S*)mdl.mu; md.delta = (const S*)mdl.delta; md.xhat0 = (const S*)mdl.xhat0;
    md.gamma = mdl.gamma;
    SqpWork<S> w;
    S** slots[19] = {&w.A, &w.B, &w.c, &w.x0, &w.Ex, &w.Eu, &w.e, &w.W, &w.Gx, &w.Gu, &w.g,
                     &w.Q, &w.M, &w.R, &w.q, &w.r, &w.dx, &w.du, &w.lqp};
    for (int i = 0; i < 19; ++i) *slots[i] = (S*)(ws + l.off[i]);
    w.th = (double*)(ws + l.off[19]);
    w.J = (double*)(ws + l.off[20]);
    w.dJ = (double*)(ws + l.off[21]);
    const int64_t B = mdl.batch;
    const int N = mdl.N, n = mdl.n, m = mdl.m, nc = mdl.nc, p = n + m;
    const size_t es = sizeof(S);
    const Tuning* tun = h->find(B, N, n, m, o.dtype);
    LCHK(launch_nt(64, F_SQP, 0, 0, k_sqp_setup<S>, B * (N + 1), s, md, w));
    QpArgs<S> qa{B, N, n, m, p, nc, w.Ex, w.Eu, w.e, w.W, w.Gx, w.Gu, w.g, md.mu, md.delta,
                 w.Q, w.M, w.R, w.q, w.r};
    const size_t qlds = es * ((size_t)p * (n + m) + p + 2 * (size_t)nc);
    for (int it = 0; it < iters; ++it) {
        LCHK(launch_nt(64, F_SQP, 0, 0, k_sqp_linearize<S>, B * (N + 1), s, md, w, (const S*)X, (const S*)U));
        hipLaunchKernelGGL(k_qp_build<S>, dim3((unsigned)(B * (N + 1))), dim3(256), qlds, s, qa);
        HIPCHK(hipGetLastError());
        LCHK(solve_impl(h, s, B, N, n, m, w.A, w.B, w.c, w.Q, w.R, w.M, w.q, w.r, w.x0, w.dx, w.du, w.lqp, status,
                        ws + l.solve_off, ws_bytes - l.solve_off, o, tun));
        LCHK(launch_nt(64, F_SQP, 0, 0, k_sqp_trials<S>, B * (kAlphas + 1), s, md, w, (const S*)X, (const S*)U));
        LCHK(launch_nt(64, F_SQP, 0, 0, k_sqp_update<S>, B, s, md, w, X, U, L,
                       alpha_out ? alpha_out + (int64_t)it * B : (S*)nullptr, status, theta_max, 1e-4));
    }
    return LQR_OK;
}
}  // namespace

extern "C" {

int lqr_sqp_workspace_size(lqr_handle_t h, int64_t batch, int N, int n, int m, int nc, const lqr_opts* opts,
                           size_t* bytes) {
    if (!bytes) return fail(LQR_EINVAL, "null output pointer");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    LCHK(sqp_check(batch, N, n, m, nc, o));
    *bytes = sqp_layout(h, batch, N, n, m, nc, o).total;
    return LQR_OK;
}

int lqr_sqp_solve(lqr_handle_t h, void* stream, const lqr_bilinear_model* mdl, int iters, double theta_max, void* x,
                  void* u, void* lam, void* alpha_out, int32_t* status, void* workspace, size_t workspace_bytes,
                  const lqr_opts* opts) {
    if (!h || !mdl) return fail(LQR_EINVAL, "null handle or model");
    lqr_opts o;
    if (opts) o = *opts; else lqr_opts_default(&o, LQR_F32);
    LCHK(sqp_check(mdl->batch, mdl->N, mdl->n, mdl->m, mdl->nc, o));
    if (iters < 0 || iters > 1000) return fail(LQR_EINVAL, "iters must be in 0..1000");
    if (!(theta_max >= 0.0)) return fail(LQR_EINVAL, "theta_max must be >= 0");
    const size_t es = o.dtype == LQR_F32 ? 4 : 8;
    const void* need[] = {mdl->A, mdl->B, mdl->c, mdl->P, mdl->V, mdl->xr, mdl->ur, mdl->wx, mdl->wu, mdl->xhat0,
                          x, u, lam, status, workspace};
    for (const void* ptr : need)
        if (!ptr) return fail(LQR_EINVAL, "null pointer argument");
    if (mdl->nc > 0 && (!mdl->Gx || !mdl->Gu || !mdl->g0 || !mdl->mu || !mdl->delta))
        return fail(LQR_EINVAL, "null constraint array");
    if (!aligned(workspace, 256) || !aligned(x, es) || !aligned(u, es) || !aligned(lam, es))
        return fail(LQR_EINVAL, "misaligned argument");
    const SqpLayout l = sqp_layout(h, mdl->batch, mdl->N, mdl->n, mdl->m, mdl->nc, o);
    if (workspace_bytes < l.total)
        return fail(LQR_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", workspace_bytes, l.total);
    HIPCHK(hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    o.sync_status = 0;
    int rc;
    {
        TimerScope ts_scope(h->timing ? &h->timer : nullptr);
        rc = o.dtype == LQR_F32
                 ? sqp_run<float>(h, s, *mdl, iters, theta_max, (float*)x, (float*)u, (float*)lam, (float*)alpha_out,
                                  status, (char*)workspace, workspace_bytes, l, o)
                 : sqp_run<double>(h, s, *mdl, iters, theta_max, (double*)x, (double*)u, (double*)lam,
                                   (double*)alpha_out, status, (char*)workspace, workspace_bytes, l, o);
    }
    if (rc != LQR_OK || !(opts && opts->sync_status)) return rc;
    return sync_status_check(s, status, mdl->batch);
}

int lqr_timing_enable(lqr_handle_t h, int enable) {
    if (!h) return fail(LQR_EINVAL, "null handle");
    h->timing = enable != 0;
    return LQR_OK;
}

int lqr_timing_report(lqr_handle_t h, char* buf, size_t len) {
    if (!h || !buf || len == 0) return fail(LQR_EINVAL, "null handle or buffer");
    HIPCHK(hipSetDevice(h->device));
    struct Acc { int64_t launches = 0; double ms = 0, flops = 0, bytes = 0, flops_min = 0; } acc[F_COUNT];
    for (auto& r : h->timer.recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        Acc& a = acc[r.fam];
        a.launches += 1;
        a.ms += ms;
        a.flops += r.flops;
        a.bytes += r.bytes;
        a.flops_min += r.flops_min;
        h->timer.pool.push_back(r.a);
        h->timer.pool.push_back(r.b);
    }
    h->timer.recs.clear();
    std::string out;
    char line[256];
    for (int f = 0; f < F_COUNT; ++f) {
        if (!acc[f].launches) continue;
        snprintf(line, sizeof line, "%s %lld %.6f %.6e %.6e %.6e\n", kFamNames[f], (long long)acc[f].launches,
                 acc[f].ms, acc[f].flops, acc[f].bytes, acc[f].flops_min);
        out += line;
    }
    if (out.size() + 1 > len) return fail(LQR_ENOMEM, "report needs %zu bytes", out.size() + 1);
    std::memcpy(buf, out.c_str(), out.size() + 1);
    return LQR_OK;
}

}  // extern "C"
