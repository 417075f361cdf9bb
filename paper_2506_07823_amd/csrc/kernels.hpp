// kernels.hpp -- HIP kernels of the LQR-KKT solve (gfx950).
//
// Paper: Amatucci, Sousa-Pinto et al., "Primal-Dual iLQR for GPU-Accelerated
// Learning and Control in Legged Robots" (arXiv 2506.07823), Sec. II.
//
// Kernels of the scan path, in launch order:
//   k_element   one-stage conditional value function, eq. (initialization)
//   k_up        up-sweep of the reverse scan: node = left (x) right, with the
//               combine of eq. (combination_rule) in Cholesky form
//   k_root/k_down  down-sweep: complete suffixes e_k (x) ... (x) e_N, whose
//               (P, p) is the value function (P_k, p_k) (Sec. II-D)
//   k_policy    K_k, k_k of eq. (lqr) from P_{k+1}, p_{k+1}, and the
//               closed-loop map (Abar_k, bbar_k) of eq. (controlled_dynamics)
//   k_fup/k_fdown  parallel scan of the closed-loop affine maps: up-sweep
//               composes maps, down-sweep pushes the initial state to every
//               node (Sec. II-D, conditional optimal trajectories)
//   k_recover   u_k = K_k x_k + k_k, lambda_k = P_k x_k + p_k (Sec. II-C)
// Refinement (one sweep): k_resid (FP64 KKT residual) -> k_ref_d ->
// k_bvec_up/k_bvec_down (backward affine scan of the gradient recursion with
// the stored closed-loop products) -> k_ref_kff -> k_fvec_up/k_fdown ->
// k_recover<ADD>.
// Plain baseline: k_plain runs the sequential Riccati sweep of eq. (lqr).
//
// One 64-lane group (G = 8) owns one task; E::TS selects the padded order.
#pragma once
#include "bigeng.hpp"
#include "engine.hpp"

namespace lqr {

#define LQR_MAXLEV 24

struct Tree {
    int nlev, total;
    int cnt[LQR_MAXLEV];
    int off[LQR_MAXLEV];
};

struct Plan {
    int64_t batch;
    int N, n, m;
    int rec, srec, frec;   // record sizes (elements): tree node, suffix, forward node
    Tree rt, ft;           // reverse tree over N+1 leaves, forward tree over N leaves
    int64_t stride;        // elements of the storage type per instance
    int64_t o_tree, o_suf, o_K, o_kff, o_LG, o_ftree, o_xs, o_w, o_pend;
    int64_t o_cp, o_qp, o_rp, o_x0p, o_pp, o_kffp;
    int64_t dstride;       // doubles per instance: partial norms 2*(N+1)
    double cond_thr;
    double refine_tol;
    int fallback;
    const int32_t* active;   // refinement gating: instances with active[b] == 0 skip (nullptr = all)
    int fused;               // 1: per-instance kernels for the vector-only passes
    int sched;               // reverse scan: 0 balanced tree over all N+1 leaves; 1 split (tree over
                             // [0, tail), tail a power of two); 2 chunked (chunks of `chunk` leaves
                             // over [0, tail)); in 1 and 2 a sequential sweep covers [tail, N]
    int tail;                // first leaf of the sequential sweep (schedules 1 and 2)
    int chunk;               // chunk length (schedule 2)
    int nchunk;              // chunks over [0, tail) (schedule 2)
    int fwdseq;              // 1: forward scan and refinement vector passes as sequential sweeps
                             // over the stages, one task unit per instance
    int64_t o_V;             // V_k' = L_R^{-1} B_k' (m x n) of the leaves k < N, for the low-rank
                             // leaf combine of the sequential sweeps (-1: no such section)
    int leafv;               // 1: the elements store V_k' and the chunked schedule's sweeps
                             // combine leaves through it (leaf_combine)
    int noC;                 // 1: no combine reads a leaf's C (every leaf goes through V), so the
                             // elements leave that part of their records unwritten
    int fuse_elem;           // 1: the chunk-1 sweep builds each leaf itself (k_chunk_mid_elem):
                             // no element launch, no leaf records
    int64_t o_scr;           // large-block engine: byte offset of the per-workgroup scratch area
    int64_t scr_elems;       //   its elements per workgroup
    int big_grid;            //   workgroups of a task launch (scratch slots)
};

// Balanced tree over `leaves` nodes, level by level (a level of c nodes has
// ceil(c / 2) parents; an odd last node is carried up)
__host__ __device__ inline Tree make_tree(int leaves) {
    Tree t{};
    t.nlev = 1;
    t.cnt[0] = leaves;
    t.off[0] = 0;
    t.total = leaves;
    while (t.cnt[t.nlev - 1] > 1) {
        t.cnt[t.nlev] = (t.cnt[t.nlev - 1] + 1) / 2;
        t.off[t.nlev] = t.total;
        t.total += t.cnt[t.nlev];
        ++t.nlev;
    }
    return t;
}

__host__ __device__ inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Shapes whose sequential sweeps combine each leaf through its rank-m factor
// (wavefront-engine orders 17..64 with m <= 16: an m x m factorization in
// place of two n x n ones)
__host__ __device__ inline bool leaf_lowrank(int n, int m) { return m <= 16 && n > 16 && n <= 64; }

// Per-instance record layout of a scan solve of shape (N, n, m), in elements
// of the storage type (every section 64-element aligned):
//   tree  reverse-scan nodes (A, C, P, b, p)       suf   complete suffixes (P, p)
//   K, kff, LG  policy and its Cholesky factor      ftree forward-scan nodes (M, v)
//   xs, w, pend  node vectors of the vector scans   cp .. kffp  refinement data
//   V     the leaves' rank-m factors (leaf_lowrank shapes only)
__host__ __device__ inline void plan_records(Plan& p, int N, int n, int m, bool with_v = true) {
    p.N = N; p.n = n; p.m = m;
    const int64_t nn = (int64_t)n * n;
    p.rec = (int)(3 * nn + 2 * n);
    p.srec = (int)(nn + n);
    p.frec = (int)(nn + n);
    p.rt = make_tree(N + 1);
    p.ft = make_tree(N);
    int64_t off = 0;
    auto sec = [&](int64_t count) { const int64_t o = off; off = align_up(off + count, 64); return o; };
    p.o_tree = sec((int64_t)p.rt.total * p.rec);
    p.o_suf = sec((int64_t)p.rt.total * p.srec);
    p.o_K = sec((int64_t)N * m * n);
    p.o_kff = sec((int64_t)N * m);
    p.o_LG = sec((int64_t)N * m * m);
    p.o_ftree = sec((int64_t)p.ft.total * p.frec);
    p.o_xs = sec((int64_t)p.ft.total * n);
    p.o_w = sec((int64_t)p.ft.total * n);
    p.o_pend = sec((int64_t)p.ft.total * n);
    p.o_cp = sec((int64_t)N * n);
    p.o_qp = sec((int64_t)(N + 1) * n);
    p.o_rp = sec((int64_t)N * m);
    p.o_x0p = sec(n);
    p.o_pp = sec((int64_t)(N + 1) * n);
    p.o_kffp = sec((int64_t)N * m);
    p.o_V = with_v && leaf_lowrank(n, m) ? sec((int64_t)N * m * n) : -1;
    p.leafv = 0;
    p.noC = 0;
    p.fuse_elem = 0;
    p.stride = off;
    p.dstride = 2 * (N + 1);
}

// Layout of one FP64 redo slot (the sequential recursion's P_k, p_k by stage,
// K_k, k_k), in doubles: sets o_suf, o_K, o_kff, stride of r
__host__ __device__ inline void redo_records(Plan& r) {
    int64_t off = 0;
    auto sec = [&](int64_t count) { const int64_t o = off; off = align_up(off + count, 64); return o; };
    r.o_suf = sec((int64_t)(r.N + 1) * r.srec);
    r.o_K = sec((int64_t)r.N * r.m * r.n);
    r.o_kff = sec((int64_t)r.N * r.m);
    r.stride = off;
}

#define LQR_GATE(p, b) \
    do {               \
        if ((p).active && !(p).active[(b)]) return; \
    } while (0)

template <typename S>
struct In {
    const S *A, *B, *c, *Q, *R, *M, *q, *r, *x0;
};

template <typename S>
struct Out {
    S *x, *u, *lam;
    int32_t* status;
};

// optional warm start of the scan (null x: cold start)
template <typename S>
struct Warm {
    const S *x, *u, *lam;
};

// pointer helpers (instance b, stage k)
template <typename S> struct Ptr {
    const Plan& p;
    const In<S>& in;
    __device__ Ptr(const Plan& p_, const In<S>& in_) : p(p_), in(in_) {}
    __device__ const S* A(int64_t b, int k) const { return in.A + ((b * p.N + k) * p.n) * p.n; }
    __device__ const S* B(int64_t b, int k) const { return in.B + ((b * p.N + k) * p.n) * p.m; }
    __device__ const S* c(int64_t b, int k) const { return in.c + (b * p.N + k) * p.n; }
    __device__ const S* Q(int64_t b, int k) const { return in.Q + ((b * (p.N + 1) + k) * p.n) * p.n; }
    __device__ const S* R(int64_t b, int k) const { return in.R + ((b * p.N + k) * p.m) * p.m; }
    __device__ const S* M(int64_t b, int k) const { return in.M + ((b * p.N + k) * p.n) * p.m; }
    __device__ const S* q(int64_t b, int k) const { return in.q + (b * (p.N + 1) + k) * p.n; }
    __device__ const S* r(int64_t b, int k) const { return in.r + (b * p.N + k) * p.m; }
    __device__ const S* x0(int64_t b) const { return in.x0 + b * p.n; }
};

__device__ __forceinline__ int suffix_id(const Tree& t, int l, int j) {
    while (l < t.nlev - 1 && (j & 1) == 0) { j >>= 1; ++l; }
    return t.off[l] + j;
}

// Tasks of a reverse-tree launch.  Under the split schedule only the nodes
// whose leaves all lie in [0, tail) are combined (tail is a power of two, so
// no node straddles the boundary); the suffixes of leaves >= tail come from
// the sequential sweep.
__host__ __device__ __forceinline__ int up_count(const Plan& p, int lvl) {
    return p.sched == 1 ? (p.tail >> (lvl + 1)) : p.rt.cnt[lvl + 1];
}
__host__ __device__ __forceinline__ int down_half(const Plan& p, int lvl) {
    return p.sched == 1 ? (p.tail >> lvl) / 2 : p.rt.cnt[lvl] / 2;
}

template <class E>
struct Lds {
    using T = typename E::T;
    T sA[E::MAT];
    T sX[E::MAT];
    T vb[E::NP];   // staged vector of the matrix-vector products
    T cb[1];    // (the factorization and solves hand pivots over
    T rb[1];    //  in registers)
};

template <typename T>
struct Lds<BigEng<T>> : BigLds<T> {};

// Wavefronts per SIMD that the two-slot LDS of a one-wavefront workgroup
// allows (160 KiB per CU, 4 SIMDs): the register budget a kernel gets
// without costing occupancy, passed as its launch bound's minimum
template <class E>
constexpr int lds_waves_per_simd() {
    constexpr int w = ((int)(163840 / sizeof(Lds<E>)) + 3) / 4;   // the fullest SIMD
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// Launch bound of the FP32 sweeps of cheap combines (k_chunk_mid,
// k_chunk_down, k_tail): where their two LDS matrix slots hold occupancy to
// 3 wavefronts per SIMD or fewer, the register budget of that occupancy, so
// that the batched slot copies of the cheap combine do not cost a wavefront;
// otherwise no bound
template <class E>
constexpr int combine_min_waves() {
    constexpr int w = lds_waves_per_simd<E>();
    return (sizeof(typename E::T) == 4 && w <= 3) ? w : 1;
}

// LDS of the vector-only passes: two staging vectors (nothing else, so these
// kernels keep many wavefronts resident to hide their memory latency)
template <class E>
struct VecLds {
    typename E::T vb[2][E::NP];
};

template <class E>
struct ResidLds {
    double vb[3][E::NP];
};

template <class E>
struct Lds3 : Lds<E> {
    typename E::T sP[E::MAT];
};

// Task units.  A task runs on NTU threads (a power of two): one wavefront
// (64) for the wavefront engine, the whole 256-thread workgroup for the
// large-block engine.  NTU = 0 means the whole workgroup.  The fused solve
// runs several wavefront tasks side by side in one workgroup, so the task
// bodies use the unit-relative thread index.
template <int NTU>
__device__ __forceinline__ int unit_tid() { return NTU ? (int)(threadIdx.x & (NTU - 1)) : (int)threadIdx.x; }
template <int NTU>
__device__ __forceinline__ int unit_nt() { return NTU ? NTU : (int)blockDim.x; }

// strided cooperative copy of `count` elements (every thread of the task
// unit; element i < unit size is handled by thread i)
template <int NTU = 0, typename D, typename S>
__device__ __forceinline__ void coop_copy(D* dst, const S* src, int count) {
    for (int i = unit_tid<NTU>(); i < count; i += unit_nt<NTU>()) dst[i] = D(src[i]);
}
template <int NTU = 0, typename D>
__device__ __forceinline__ void coop_zero(D* dst, int count) {
    for (int i = unit_tid<NTU>(); i < count; i += unit_nt<NTU>()) dst[i] = D(0);
}

// load a rows x cols global matrix (optionally transposed) into an LDS slot
template <class E, bool TR = false, typename S>
__device__ __forceinline__ void stage(const E& e, typename E::T* slot, const S* g, int rows, int cols, int ldg) {
    if (!TR) {
        e.g2s_batched(slot, g, rows, cols, ldg);
    } else {
        typename E::Tile t;
        e.template load<TR>(t, g, rows, cols, ldg);
        e.to_lds(t, slot);
    }
}

template <class E>
__device__ __forceinline__ void to_lds_sym(const E& e, const typename E::Tile& t, typename E::T* s) {
    e.to_lds_sym(t, s);
}

template <class E>
__device__ __forceinline__ void negate(typename E::Tile& t) {
#pragma unroll
    for (int a = 0; a < E::TS; ++a)
#pragma unroll
        for (int b = 0; b < E::TS; ++b) t[a][b] = -t[a][b];
}

// reciprocal diagonal of a staged lower-triangular factor

template <int NTU = 0>
__device__ __forceinline__ void set_status(int32_t* status, int64_t b, int bits) {
    if (unit_tid<NTU>() == 0) atomicOr(status + b, bits);
}


// ---------------------------------------------------------------------------
// FP64 fallback.  An FP32 task whose Cholesky factorization fails or whose
// condition estimate (max L_ii / min L_ii)^2 exceeds the threshold marks its
// instance (status bit 8).  Once the FP32 launch sequence has finished, the
// marked instances are solved again whole with FP64 arithmetic and FP64
// intermediates (k_redo): FP32 records of such an instance (the element of
// an ill-conditioned R_k has eigenvalues spread over the square of its
// condition number) cannot be repaired by redoing one factorization.
// Without the fallback a failed factorization sets `failbit` instead.
// ---------------------------------------------------------------------------
template <int NTU = 0, typename T>
__device__ __forceinline__ void fb_flag(const Plan& p, bool ok, T kappa, int64_t b, int32_t* status, int failbit) {
    const bool bad = !ok || !(kappa <= T(p.cond_thr));
    if (!bad) return;
    if (p.fallback) set_status<NTU>(status, b, 8);
    else if (!ok) set_status<NTU>(status, b, failbit);
}

template <typename T>
__device__ __forceinline__ T cond_est(T dmin, T dmax) {
    return dmin > T(0) ? (dmax / dmin) * (dmax / dmin) : T(3.0e38);
}

// clear the status words (a fill kernel, safe under graph capture)
template <typename I>
__global__ void k_clear(I* status, int64_t batch) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < batch) status[i] = 0;
}

// Value function and policy of the last scan solve, read back from the
// records of the workspace (one workgroup per instance and stage):
// P [b][k] (n x n), p [b][k] (n) for k = 0..N; K [b][k] (m x n), kff [b][k]
// (m) for k < N.
template <typename S>
__global__ void k_factors(Plan p, const S* ws, S* P, S* pv, S* K, S* kff) {
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = blockIdx.x / (N + 1);
    const int k = (int)(blockIdx.x % (N + 1));
    const S* inst = ws + b * p.stride;
    const S* rec = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
    const int64_t bk = b * (N + 1) + k;
    for (int i = threadIdx.x; i < nn; i += blockDim.x) P[bk * nn + i] = rec[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) pv[bk * n + i] = rec[nn + i];
    if (k == N) return;
    const int64_t bq = b * N + k;
    for (int i = threadIdx.x; i < m * n; i += blockDim.x) K[bq * m * n + i] = inst[p.o_K + (int64_t)k * m * n + i];
    for (int i = threadIdx.x; i < m; i += blockDim.x) kff[bq * m + i] = inst[p.o_kff + (int64_t)k * m + i];
}

// dst = src, count elements (grid-stride)
template <typename S>
__global__ void k_copy(const S* src, S* dst, int64_t count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// Run `body(task)` for every task of the launch: one task per workgroup, or
// grid-stride over the per-workgroup scratch slots of the large-block engine.
#define LQR_TASKS(E, ntasks, body)                                            \
    do {                                                                      \
        if (E::BIG) {                                                         \
            for (int64_t t_ = blockIdx.x; t_ < (ntasks); t_ += gridDim.x) {   \
                body(t_);                                                     \
                E::sync();                                                    \
            }                                                                 \
        } else {                                                              \
            body((int64_t)blockIdx.x);                                        \
        }                                                                     \
    } while (0)

}  // namespace lqr
#include "kernels_big.hpp"
namespace lqr {

// MB (kernel template parameter of the element, policy and plain kernels
// of the wavefront engine): the number of G-row blocks the control
// dimension m occupies, so the tile products, Cholesky and solves of
// m-sized operands skip the padding blocks.  The host picks 1, 2 or TS.


// ---------------------------------------------------------------------------
// Sec. II-D, eq. (initialization): one-stage element with S_k = M_k'.
//   R = L_R L_R',  W_B = L_R^{-1} B',  W_M = L_R^{-1} M',  w_r = L_R^{-1} r
//   At = A - W_B' W_M,  Ct = W_B' W_B,  Pt = Q - W_M' W_M,
//   bt = c - W_B' w_r,  pt = q - W_M' w_r.
// The terminal element (k = N) is (0, 0, 0, Q_N, q_N).  A factorization of
// R_k with a non-positive pivot or a condition estimate above the threshold
// marks the instance for the FP64 redo.
// Record layout: A | C | P | b | p (C left unwritten under p.noC).
// ---------------------------------------------------------------------------
template <typename S, class E, int MB>
__device__ __forceinline__ void element_task(Lds<E>& L, const Plan& p, const In<S>& in, S* ws, int32_t* status,
                             int64_t task) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = task / (N + 1);
    const int k = (int)(task % (N + 1));
    S* rec = ws + b * p.stride + p.o_tree + (int64_t)k * p.rec;
    const Ptr<S> P(p, in);
    if (k == N) {
        coop_zero<E::NT>(rec, 2 * nn);
        coop_copy<E::NT>(rec + 2 * nn, P.Q(b, N), nn);
        coop_zero<E::NT>(rec + 3 * nn, n);
        coop_copy<E::NT>(rec + 3 * nn + n, P.q(b, N), n);
        return;
    }
    typename E::Tile tR;
    e.load(tR, P.R(b, k), m, m, m);
    // loaded before the factorization (its wave barrier keeps later loads
    // from moving up), so their latency overlaps it; A, Q, c, q too (the
    // LDS already holds the kernel to 3 wavefronts per SIMD, whose register
    // budget has room for them)
    typename E::Tile W[2];
    e.template load<true>(W[0], P.B(b, k), m, n, m);   // B' (m x n)
    e.template load<true>(W[1], P.M(b, k), m, n, m);   // M' (m x n)
    T vv[1] = {e.vload(P.r(b, k), m)};
    typename E::Tile tA, tQ;
    e.load(tA, P.A(b, k), n, n, n);
    e.load(tQ, P.Q(b, k), n, n, n);
    const T cpre = e.vload(P.c(b, k), n), qpre = e.vload(P.q(b, k), n);
    T dmin, dmax, nov[1];
    T dlA;
    const bool ok = e.template chol<0, MB>(tR, m, L.cb, dlA, nov, dmin, dmax);
    fb_flag<E::NT>(p, ok, cond_est(dmin, dmax), b, status, 2);
    e.to_lds(tR, L.sA);
    wg_sync();
    e.template trsm<true, 2, 1, MB>(L.sA, dlA, m, W, vv, L.rb);
    e.to_lds(W[0], L.sA);
    e.to_lds(W[1], L.sX);
    wg_sync();
    // C_t = V V' with V = W_B' (n x m): the leaf combine of the sweeps uses V
    if (p.leafv) e.s2g(L.sA, ws + b * p.stride + p.o_V + (int64_t)k * m * n, m, n, n);
    e.template gemm_sub<true, false>(tA, L.sA, L.sX, m);
    e.store(tA, rec, n, n, n);                         // At
    if (!p.noC) {
        typename E::Tile t;
        e.zero(t);
        e.template gemm<true, false, true>(t, L.sA, L.sA, m);
        e.store_sym(t, rec + nn, n);                   // Ct
    }
    e.template gemm_sub<true, false, true>(tQ, L.sX, L.sX, m);
    e.store_sym(tQ, rec + 2 * nn, n);                  // Pt
    const T bw = e.template matvec<true>(L.sA, L.vb, vv[0], m, n);
    e.vstore(rec + 3 * nn, n, cpre - bw);
    const T pw = e.template matvec<true>(L.sX, L.vb, vv[0], m, n);
    e.vstore(rec + 3 * nn + n, n, qpre - pw);
}

template <typename S, class E, int MB>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_element(Plan p, In<S> in, S* ws, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) {
        if constexpr (E::BIG) big_element_task<S, E>(L, p, in, ws, status, t);
        else element_task<S, E, MB>(L, p, in, ws, status, t);
    };
    LQR_TASKS(E, p.batch * (p.N + 1), body);
}

// ---------------------------------------------------------------------------
// Sec. II-D, eq. (combination_rule), e1 (x) e2 with e1 the earlier segment.
// With P2 = L L', S = I + L' C1 L = L_S L_S':
//   Y = L_S^{-1} L' A1,  Z1 = L^{-1} A2',  Z = L_S^{-1} Z1
//   w1 = L_S^{-1}(L^{-1} p2 + L' b1),  w2 = L_S^{-1} L'(b1 - C1 p2)
//   P = Y'Y + P1,   p = Y'w1 + p1,   A = Z'Y,
//   C = Z1'Z1 - Z'Z + C2,   b = Z'w2 + b2.
// (equal to A2 (I+C1P2)^{-1} A1, A2 (I+C1P2)^{-1} C1 A2' + C2, ... since
// (I + C1 P2)^{-1} = L^{-T} S^{-1} L').  CHEAP: e2 is a complete suffix
// (A2 = C2 = b2 = 0), only P and p are formed and written to a suffix record.
// ---------------------------------------------------------------------------
// Sequential sweeps carry the suffix from one cheap combine to the next
// (carry != nullptr): the combine leaves P in slot sA (staged there for its
// store) and p in *carry, and a following call with P2 == nullptr takes
// them from there instead of reading back what was just stored (the same
// values: an FP32 store and load are exact, padding included).
template <class E, bool CHEAP, bool BATCH = false, typename S>
__device__ __forceinline__ void combine(const E& e, Lds<E>& L, int n, const S* e1, const S* P2, const S* p2v,
                                        const S* e2, S* outA, S* outC, S* outP, S* outb, S* outp, bool& okp,
                                        typename E::T& kappa, typename E::T* carry = nullptr) {
    using T = typename E::T;
    const int nn = n * n;
    typename E::Tile tS;
    T dmin, dmax;
    // Cheap form: A1, P1, b1, p1 go to registers up front, so their global
    // latency overlaps the two factorizations (the wave barriers keep loads
    // written at their point of use from moving up).  The general form
    // keeps them at their point of use: 50 more VGPRs there would cost a
    // wavefront per SIMD.
    typename E::Tile tA1, tP1;
    T b1pre = T(0), p1pre = T(0);
    // L = chol(P2), g = L^{-1} p2
    // BATCH (the FP32 sequential sweeps of cheap combines): the slot copies
    // issue their loads in groups, one wait per group (more registers, which
    // those kernels' launch bound budgets)
    // In the sweeps (BATCH), C1 is loaded to registers before the first
    // factorization and staged after it, A1 / P1 loaded after it: both
    // factorizations then overlap outstanding loads.
    typename E::Tile tC1;
    if constexpr (BATCH) {
        if (P2) e.g2s_batched(L.sA, P2, n, n, n);
        e.load(tC1, e1 + nn, n, n, n);
    } else {
        if (P2) e.g2s(L.sA, P2, n, n, n);
        e.g2s(L.sX, e1 + nn, n, n, n);
    }
    if constexpr (CHEAP && !BATCH) {
        e.load(tA1, e1, n, n, n);
        e.load(tP1, e1 + 2 * nn, n, n, n);
        b1pre = e.vload(e1 + 3 * nn, n);
        p1pre = e.vload(e1 + 3 * nn + n, n);
    }
    T g[1] = {P2 ? e.vload(p2v, n) : *carry};
    const T p2l = g[0];
    wg_sync();
    e.from_lds(tS, L.sA);
    T dlA, dlB;
    bool ok = e.template chol<1>(tS, n, L.cb, dlA, g, dmin, dmax);
    T kap = cond_est(dmin, dmax);
    e.to_lds(tS, L.sA);                                   // sA = L
    if constexpr (BATCH) {
        e.to_lds(tC1, L.sX);                              // sX = C1
        e.load(tA1, e1, n, n, n);
        e.load(tP1, e1 + 2 * nn, n, n, n);
        b1pre = e.vload(e1 + 3 * nn, n);
        p1pre = e.vload(e1 + 3 * nn + n, n);
    }
    wg_sync();
    T cp = T(0);
    if (!CHEAP) cp = e.template matvec<false>(L.sX, L.vb, p2l, n, n);   // C1 p2
    e.zero(tS);
    e.template gemm_tri<false, false, false, 1>(tS, L.sX, L.sA, n);   // W = C1 L (L lower)
    wg_sync();
    e.to_lds(tS, L.sX);                                   // sX = W
    wg_sync();
    e.zero(tS);
    e.template gemm_tri<true, false, true, 2>(tS, L.sA, L.sX, n);     // L' W (lower part; L' upper)
    e.add_identity(tS, n);
    T nov[1];
    ok = e.template chol<0>(tS, n, L.cb, dlB, nov, dmin, dmax) && ok;   // tS = L_S
    {
        const T ks = cond_est(dmin, dmax);
        kap = ks > kap ? ks : kap;
    }
    typename E::Tile YZ[2];
    typename E::Tile tC;
    if (!CHEAP) {
        e.g2s(L.sX, e2, n, n, n);                         // A2
        wg_sync();
        typename E::Tile Z1[1];
        e.from_lds_t(Z1[0], L.sX);                        // A2'
        e.template trsm<true, 1, 0>(L.sA, dlA, n, Z1, nov, L.rb);   // Z1 = L^{-1} A2'
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int bb = 0; bb < E::TS; ++bb) YZ[1][a][bb] = Z1[0][a][bb];
    }
    if constexpr (CHEAP) e.to_lds(tA1, L.sX);             // sX = A1
    else e.g2s(L.sX, e1, n, n, n);
    wg_sync();
    e.zero(YZ[0]);
    e.template gemm_tri<true, false, false, 2>(YZ[0], L.sA, L.sX, n); // L' A1 (L' upper)
    const T b1 = CHEAP ? b1pre : e.vload(e1 + 3 * nn, n);
    T vv[2];
    vv[0] = g[0] + e.template matvec<true>(L.sA, L.vb, b1, n, n);
    wg_sync();
    if (!CHEAP) {
        vv[1] = e.template matvec<true>(L.sA, L.vb, b1 - cp, n, n);
        wg_sync();
        e.to_lds(YZ[1], L.sX);                             // sX = Z1
        wg_sync();
        e.zero(tC);
        e.template gemm<true, false, true>(tC, L.sX, L.sX, n);   // Z1' Z1 (lower)
    } else {
        vv[1] = T(0);
    }
    wg_sync();
    e.to_lds(tS, L.sA);                                    // sA = L_S
    wg_sync();
    if (!CHEAP) {
        e.template trsm<true, 2, 2>(L.sA, dlB, n, YZ, vv, L.rb);
    } else {
        typename E::Tile Y1[1];
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int bb = 0; bb < E::TS; ++bb) Y1[0][a][bb] = YZ[0][a][bb];
        T v1[1] = {vv[0]};
        e.template trsm<true, 1, 1>(L.sA, dlB, n, Y1, v1, L.rb);
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int bb = 0; bb < E::TS; ++bb) YZ[0][a][bb] = Y1[0][a][bb];
        vv[0] = v1[0];
    }
    e.to_lds(YZ[0], L.sX);                                 // sX = Y
    if constexpr (CHEAP) {
        wg_sync();
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int bb = 0; bb < E::TS; ++bb) tS[a][bb] = tP1[a][bb];   // P1
    } else {
        e.g2s(L.sA, e1 + 2 * nn, n, n, n);                 // sA = P1
        wg_sync();
        e.from_lds(tS, L.sA);
    }
    e.template gemm<true, false, true>(tS, L.sX, L.sX, n); // P1 + Y'Y (lower)
    const T pv = e.template matvec<true>(L.sX, L.vb, vv[0], n, n) + (CHEAP ? p1pre : e.vload(e1 + 3 * nn + n, n));
    e.vstore(outp, n, pv);
    if (carry) *carry = pv;
    wg_sync();
    e.to_lds_sym(tS, L.sA);                                // sA = P
    wg_sync();
    e.s2g(L.sA, outP, n, n, n);
    if (!CHEAP) {
        wg_sync();
        e.to_lds(YZ[1], L.sA);                             // sA = Z
        wg_sync();
        e.zero(tS);
        e.template gemm<true, false>(tS, L.sA, L.sX, n);   // A = Z'Y
        e.template gemm_sub<true, false, true>(tC, L.sA, L.sA, n);   // Z1'Z1 - Z'Z (lower)
        const T bv = e.template matvec<true>(L.sA, L.vb, vv[1], n, n) + e.vload(e2 + 3 * nn, n);
        e.vstore(outb, n, bv);
        wg_sync();
        e.to_lds(tS, L.sX);                                // sX = A
        e.to_lds_sym(tC, L.sA);                            // sA = Z1'Z1 - Z'Z
        wg_sync();
        e.s2g(L.sX, outA, n, n, n);
        // C = sA + C2 (coalesced read-add-write)
        const float invn = 1.0f / (float)n;
        for (int idx = e.lg; idx < nn; idx += E::GL) {
            const int i = (int)(((float)idx + 0.5f) * invn), j = idx - i * n;
            outC[idx] = S(L.sA[i * E::LD + j] + T(e2[nn + idx]));
        }
    }
    wg_sync();
    okp = ok;
    kappa = kap;
}

// ---------------------------------------------------------------------------
// Cheap combine of a leaf e1 = (A1, b1, C1, P1, p1) with a complete suffix
// (P2, p2), Sec. II-D eq. (combination_rule), where C1 = V V' has rank m
// (V = B R^{-1/2}, eq. (initialization)).  By the Woodbury identity
//   (I + P2 C1)^{-1} P2 = P2 - P2 V S^{-1} V' P2,   S = I_m + V' P2 V,
// so with S = L_S L_S', U = L_S^{-1} V' P2 (m x n) and z = p2 + P2 b1:
//   P = P1 + A1' (P2 - U'U) A1,   p = p1 + A1' (z - U' L_S^{-1} V' z),
// the same (P, p) as the form above, with one m x m factorization in place
// of the two n x n ones (S >= I: its pivots are at least 1).  The products
// with an m-row operand form only the first MB row blocks.  Vt: the leaf's
// V' (m x n, row-major).  P2 == nullptr: the suffix is the one the previous
// call left in slot sA and *carry (the carry convention of combine).
// ---------------------------------------------------------------------------
// The combine proper: V' staged in the first MB row blocks of sX (the rows
// past them are left as they are), P2 in sA, the leaf's A1 (tile), b1, p1
// (lane vectors); get_p1(tile) forms the leaf's P1 (lower triangle) after
// the factorization, whose latency its loads then overlap.
template <class E, int MB, typename S, class GetP1>
__device__ __forceinline__ void leaf_core(const E& e, Lds<E>& L, int n, int m, typename E::Tile& tA1, GetP1&& get_p1,
                                          typename E::T b1, typename E::T p1, typename E::T p2, S* outP, S* outp,
                                          bool& okp, typename E::T& kappa, typename E::T* carry) {
    using T = typename E::T;
    static_assert(MB >= 1 && MB < E::TS, "m spans fewer row blocks than the order");
    typename E::Tile tM, tS, tP1;
    typename E::Tile TU[1];
    e.from_lds(tM, L.sA);                           // P2
    e.zero(TU[0]);
    e.template gemm<false, false, false, false, MB, E::TS>(TU[0], L.sX, L.sA, n);   // V' P2
    const T z = p2 + e.template matvec<false>(L.sA, L.vb, b1, n, n);                // p2 + P2 b1
    T w[1] = {e.template matvec<false>(L.sX, L.vb, z, n, m)};                       // V' z
    wg_sync();
    e.to_lds(TU[0], L.sA);                          // sA = V' P2
    wg_sync();
    e.zero(tS);
    e.template gemm<false, true, false, false, MB, MB>(tS, L.sA, L.sX, n);         // V' P2 V
    e.add_identity(tS, m);
    T dl, dmin, dmax;
    const bool ok = e.template chol<1, MB>(tS, m, L.cb, dl, w, dmin, dmax);        // L_S; w = L_S^{-1} V' z
    e.template to_lds_rows<MB>(tS, L.sX);           // sX = L_S (its MB row blocks)
    wg_sync();
    T nov[1];
    e.template trsm<true, 1, 0, MB>(L.sX, dl, m, TU, nov, L.rb);                    // U = L_S^{-1} V' P2
    get_p1(tP1);
    e.to_lds(TU[0], L.sA);                          // sA = U
    wg_sync();
    e.template gemm_sub<true, false, true>(tM, L.sA, L.sA, m);                      // P2 - U'U (lower)
    const T y = z - e.template matvec<true>(L.sA, L.vb, w[0], m, n);                // z - U' w
    wg_sync();
    e.to_lds_sym(tM, L.sX);                         // sX = M = P2 - U'U
    e.to_lds(tA1, L.sA);                            // sA = A1
    wg_sync();
    e.zero(tS);
    e.template gemm<false, false>(tS, L.sX, L.sA, n);                               // M A1
    wg_sync();
    e.to_lds(tS, L.sX);                             // sX = M A1
    wg_sync();
    e.template gemm<true, false, true>(tP1, L.sA, L.sX, n);                         // P1 + A1' M A1 (lower)
    const T pv = e.template matvec<true>(L.sA, L.vb, y, n, n) + p1;                // p1 + A1' y
    e.vstore(outp, n, pv);
    if (carry) *carry = pv;
    wg_sync();
    e.to_lds_sym(tP1, L.sA);                        // sA = P (kept for a carried call)
    wg_sync();
    e.s2g(L.sA, outP, n, n, n);
    wg_sync();
    okp = ok;
    kappa = cond_est(dmin, dmax);
}

template <class E, int MB, typename S>
__device__ __forceinline__ void leaf_combine(const E& e, Lds<E>& L, int n, int m, const S* e1, const S* Vt,
                                             const S* P2, const S* p2v, S* outP, S* outp, bool& okp,
                                             typename E::T& kappa, typename E::T* carry) {
    using T = typename E::T;
    const int nn = n * n;
    typename E::Tile tA1;
    e.load(tA1, e1, n, n, n);                       // its latency overlaps the products
    const T b1 = e.vload(e1 + 3 * nn, n);
    const T p1 = e.vload(e1 + 3 * nn + n, n);
    if (P2) e.g2s_batched(L.sA, P2, n, n, n);       // sA = P2
    // sX = V' in its first MB row blocks (zero past m and n)
    for (int idx = e.lg; idx < MB * E::G * E::NP; idx += E::GL) {
        const int i = idx / E::NP, j = idx - (idx / E::NP) * E::NP;
        L.sX[i * E::LD + j] = (i < m && j < n) ? T(Vt[i * n + j]) : T(0);
    }
    const T p2 = P2 ? e.vload(p2v, n) : *carry;
    wg_sync();
    leaf_core<E, MB>(e, L, n, m, tA1, [&](typename E::Tile& t) { e.load(t, e1 + 2 * nn, n, n, n); }, b1, p1, p2,
                     outP, outp, okp, kappa, carry);
}

// The same step with the leaf built in place from the stage inputs
// (eq. (initialization), as element_task: R = L_R L_R', [W_B; W_M] =
// L_R^{-1} [B'; M'], w_r = L_R^{-1} r, At = A - W_B'W_M, Pt = Q - W_M'W_M,
// bt = c - W_B'w_r, pt = q - W_M'w_r, V' = W_B): W_B and W_M take the two
// halves of slot sX, sA keeps the suffix, At, bt, pt stay in registers, and
// Pt is formed where the combine needs it, from W_M, which the combine
// leaves in place until then.  The same arithmetic in the same order as
// the element kernel followed by leaf_combine.
template <class E, int MB, typename S>
__device__ __forceinline__ void leaf_elem_combine(const E& e, Lds<E>& L, const Plan& p, const Ptr<S>& P, int64_t b,
                                                  int k, const S* P2, const S* p2v, S* outP, S* outp, bool& okp,
                                                  typename E::T& kappa, bool& okR, typename E::T& kappaR,
                                                  typename E::T* carry) {
    using T = typename E::T;
    static_assert(2 * MB * E::G <= E::NP, "W_B and W_M share one slot");
    const int n = p.n, m = p.m;
    T* sW = L.sX + MB * E::G * E::LD;               // W_M below V'
    typename E::Tile W[2];
    T vv[1];
    {
        typename E::Tile tR;
        e.load(tR, P.R(b, k), m, m, m);
        e.template load<true>(W[0], P.B(b, k), m, n, m);   // B'
        e.template load<true>(W[1], P.M(b, k), m, n, m);   // M'
        vv[0] = e.vload(P.r(b, k), m);
        T dmin, dmax, nov[1];
        T dlR;
        okR = e.template chol<0, MB>(tR, m, L.cb, dlR, nov, dmin, dmax);
        kappaR = cond_est(dmin, dmax);
        e.template to_lds_rows<MB>(tR, L.sX);       // L_R
        wg_sync();
        e.template trsm<true, 2, 1, MB>(L.sX, dlR, m, W, vv, L.rb);
    }
    e.template to_lds_rows<MB>(W[0], L.sX);         // V' = W_B
    e.template to_lds_rows<MB>(W[1], sW);           // W_M
    typename E::Tile tA1;
    e.load(tA1, P.A(b, k), n, n, n);
    const T cpre = e.vload(P.c(b, k), n), qpre = e.vload(P.q(b, k), n);
    if (P2) e.g2s_batched(L.sA, P2, n, n, n);       // sA = P2
    const T p2 = P2 ? e.vload(p2v, n) : *carry;
    wg_sync();
    e.template gemm_sub<true, false>(tA1, L.sX, sW, m);                             // At
    const T b1 = cpre - e.template matvec<true>(L.sX, L.vb, vv[0], m, n);           // bt
    const T p1 = qpre - e.template matvec<true>(sW, L.vb, vv[0], m, n);             // pt
    wg_sync();
    leaf_core<E, MB>(
        e, L, n, m, tA1,
        [&](typename E::Tile& t) {
            e.load(t, P.Q(b, k), n, n, n);
            e.template gemm_sub<true, false, true>(t, sW, sW, m);                   // Pt (lower)
        },
        b1, p1, p2, outP, outp, okp, kappa, carry);
}

template <typename S, class E>
__device__ __forceinline__ void up_task(Lds<E>& L, const Plan& p, S* ws, int lvl, int32_t* status, int64_t task) {
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const int cout = up_count(p, lvl), cin = p.rt.cnt[lvl];
    const int64_t b = task / cout;
    const int i = (int)(task % cout);
    S* base = ws + b * p.stride + p.o_tree;
    const S* e1 = base + (int64_t)(p.rt.off[lvl] + 2 * i) * p.rec;
    S* out = base + (int64_t)(p.rt.off[lvl + 1] + i) * p.rec;
    if (2 * i + 1 >= cin) {
        coop_copy<E::NT>(out, e1, p.rec);
        return;
    }
    const S* e2 = e1 + p.rec;
    bool ok;
    typename E::T kappa;
    combine<E, false>(e, L, n, e1, e2 + 2 * nn, e2 + 3 * nn + n, e2, out, out + nn, out + 2 * nn, out + 3 * nn,
                      out + 3 * nn + n, ok, kappa);
    fb_flag<E::NT>(p, ok, kappa, b, status, 4);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_up(Plan p, S* ws, int lvl, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) {
        if constexpr (E::BIG) big_up_task<S, E>(L, p, ws, lvl, status, t);
        else up_task<S, E>(L, p, ws, lvl, status, t);
    };
    LQR_TASKS(E, p.batch * up_count(p, lvl), body);
}

// root of the reverse tree: its (P, p) is the complete suffix starting at 0
template <typename S>
__device__ __forceinline__ void root_body(const Plan& p, S* ws, int64_t b) {
    const int n = p.n, nn = n * n;
    const int root = p.rt.off[p.rt.nlev - 1];
    const S* src = ws + b * p.stride + p.o_tree + (int64_t)root * p.rec;
    S* dst = ws + b * p.stride + p.o_suf + (int64_t)root * p.srec;
    coop_copy<64>(dst, src + 2 * nn, nn);          // P
    coop_copy<64>(dst + nn, src + 3 * nn + n, n);  // p (the record stores b between P and p)
}

template <typename S>
__global__ void k_root(Plan p, S* ws) {
    root_body<S>(p, ws, (int64_t)blockIdx.x);
}

// down-sweep at level lvl: odd node j gets node_j (x) suffix(level lvl+1, (j+1)/2)
template <typename S, class E>
__device__ __forceinline__ void down_task(Lds<E>& L, const Plan& p, S* ws, int lvl, int32_t* status, int64_t task) {
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const int half = down_half(p, lvl);
    const int64_t b = task / half;
    const int j = 2 * (int)(task % half) + 1;
    S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    const S* node = tree + (int64_t)(p.rt.off[lvl] + j) * p.rec;
    S* out = suf + (int64_t)(p.rt.off[lvl] + j) * p.srec;
    const int i1 = (j + 1) / 2;
    if (i1 >= p.rt.cnt[lvl + 1]) {
        coop_copy<E::NT>(out, node + 2 * nn, nn);
        coop_copy<E::NT>(out + nn, node + 3 * nn + n, n);
        return;
    }
    const S* s2 = suf + (int64_t)suffix_id(p.rt, lvl + 1, i1) * p.srec;
    bool ok;
    typename E::T kappa;
    combine<E, true>(e, L, n, node, s2, s2 + nn, (const S*)nullptr, (S*)nullptr, (S*)nullptr, out,
                     (S*)nullptr, out + nn, ok, kappa);
    fb_flag<E::NT>(p, ok, kappa, b, status, 4);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_down(Plan p, S* ws, int lvl, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) {
        if constexpr (E::BIG) big_down_task<S, E>(L, p, ws, lvl, status, t);
        else down_task<S, E>(L, p, ws, lvl, status, t);
    };
    LQR_TASKS(E, p.batch * down_half(p, lvl), body);
}

// ---------------------------------------------------------------------------
// Split schedule (wavefront engine).  The suffixes of the leaves >= tail are
// computed one after the other from the terminal element backwards, each as
// the combine of leaf k with the complete suffix starting at k+1 (the cheap
// form: a complete suffix has A = C = b = 0), i.e. the information form of
// the Riccati recursion of eq. (lqr).  Each is stored where the balanced
// tree would store the suffix of leaf k.  Meanwhile nothing of the tree
// depends on these leaves: the tree over [0, tail) needs only the suffix of
// leaf `tail`, taken by the root task below.  One wavefront per instance;
// the wave barrier with its fences orders each step's stores before the
// next step's loads (all lanes of the wave share one CU's caches).  A
// flagged step marks the instance for the FP64 redo.
// ---------------------------------------------------------------------------
template <typename S, class E, bool BATCH = false>
__device__ __forceinline__ void tail_task(Lds<E>& L, const Plan& p, S* ws, int32_t* status, int64_t b) {
    static_assert(!E::BIG, "wavefront engine only");
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, nn = n * n;
    S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    {
        const S* leaf = tree + (int64_t)(p.rt.off[0] + N) * p.rec;   // terminal element (0, 0, 0, Q_N, q_N)
        S* out = suf + (int64_t)suffix_id(p.rt, 0, N) * p.srec;
        coop_copy<E::NT>(out, leaf + 2 * nn, nn);
        coop_copy<E::NT>(out + nn, leaf + 3 * nn + n, n);
    }
    E::sync();
    bool ok_all = true;
    typename E::T kmax = 0;
    typename E::T pcar = 0;
    for (int k = N - 1; k >= p.tail; --k) {
        const S* node = tree + (int64_t)(p.rt.off[0] + k) * p.rec;
        const S* s2 = suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
        S* out = suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
        bool ok;
        typename E::T kappa;
        combine<E, true, BATCH>(e, L, n, node, k == N - 1 ? s2 : (const S*)nullptr, s2 + nn, (const S*)nullptr,
                                (S*)nullptr, (S*)nullptr, out, (S*)nullptr, out + nn, ok, kappa, &pcar);
        ok_all = ok_all && ok;
        if (!(kappa <= kmax)) kmax = kappa;   // NaN propagates
        E::sync();
    }
    fb_flag<E::NT>(p, ok_all, kmax, b, status, 4);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_tail(Plan p, S* ws, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) { tail_task<S, E, sizeof(typename E::T) == 4>(L, p, ws, status, t); };
    LQR_TASKS(E, p.batch, body);
}

// The sweeps and the first up-sweep level in one launch (they are
// independent): workgroups 0 .. batch-1 sweep the tails (dispatched first,
// they are the long ones), the others combine leaf pairs of the heads, so
// the combines fill the CUs while the sweeps run their dependent steps.
template <typename S, class E>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_tail_up0(Plan p, S* ws, int32_t* status) {
    static_assert(!E::BIG, "wavefront engine only");
    __shared__ Lds<E> L;
    const int64_t t = blockIdx.x;
    if (t < p.batch) tail_task<S, E>(L, p, ws, status, t);
    else up_task<S, E>(L, p, ws, 0, status, t - p.batch);
}

// Root under the split schedule: the complete suffix from leaf 0 is the
// aggregate of the head, node (nlev-2, 0), after the suffix of leaf `tail`.
template <typename S, class E>
__device__ __forceinline__ void tail_root_task(Lds<E>& L, const Plan& p, S* ws, int32_t* status,
                                               int64_t b) {
    static_assert(!E::BIG, "wavefront engine only");
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const int top = p.rt.nlev - 2;
    S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    const S* node = tree + (int64_t)p.rt.off[top] * p.rec;
    const S* s2 = suf + (int64_t)suffix_id(p.rt, 0, p.tail) * p.srec;
    S* out = suf + (int64_t)p.rt.off[p.rt.nlev - 1] * p.srec;
    bool ok;
    typename E::T kappa;
    combine<E, true>(e, L, n, node, s2, s2 + nn, (const S*)nullptr, (S*)nullptr, (S*)nullptr, out, (S*)nullptr,
                     out + nn, ok, kappa);
    fb_flag<E::NT>(p, ok, kappa, b, status, 4);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_tail_root(Plan p, S* ws, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) { tail_root_task<S, E>(L, p, ws, status, t); };
    LQR_TASKS(E, p.batch, body);
}

// ---------------------------------------------------------------------------
// Chunked schedule of the reverse scan (wavefront engine).  The leaves
// [0, tail) form `nchunk` chunks of `chunk` consecutive leaves (the last may
// be shorter); the leaves [tail, N] are swept sequentially from the terminal
// element as in the split schedule (tail_task).  Three phases:
//   1. the aggregate e_c0 (x) ... (x) e_c1-1 of every chunk, by general
//      combines from its right end (one task unit per chunk, ping-pong
//      between two records of the otherwise unused tree levels), side by
//      side with the tail sweep;
//   2. per instance, the complete suffixes at the chunk starts, from the
//      last chunk back: S_c0 = aggregate (x) S_c1, a cheap combine each;
//   3. per chunk, the complete suffixes of its other leaves from its right
//      end: S_k = e_k (x) S_k+1 (cheap).
// A chunk length of 1 over the whole horizon (tail = N) is the sequential
// information-form recursion; the balanced tree is the other extreme.  Any
// flagged step marks the instance for the FP64 redo.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int chunk_end(const Plan& p, int c) {
    const int e = (c + 1) * p.chunk;
    return e < p.tail ? e : p.tail;
}

// record holding the aggregate of chunk c (its leaf when it has one leaf)
template <typename S>
__device__ __forceinline__ const S* chunk_agg(const Plan& p, const S* tree, int c) {
    const int c0 = c * p.chunk, len = chunk_end(p, c) - c0;
    if (len == 1) return tree + (int64_t)(p.rt.off[0] + c0) * p.rec;
    return tree + (int64_t)(p.rt.off[1] + 2 * c + ((len & 1) ? 1 : 0)) * p.rec;
}

template <typename S, class E>
__device__ __forceinline__ void chunk_agg_task(Lds<E>& L, const Plan& p, S* ws, int32_t* status, int64_t b, int c) {
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    S* tree = ws + b * p.stride + p.o_tree;
    const int c0 = c * p.chunk, c1 = chunk_end(p, c);
    S* X = tree + (int64_t)(p.rt.off[1] + 2 * c) * p.rec;
    S* Y = X + p.rec;
    const S* cur = tree + (int64_t)(p.rt.off[0] + c1 - 1) * p.rec;
    bool ok_all = true;
    typename E::T kmax = 0;
    for (int k = c1 - 2, j = 0; k >= c0; --k, ++j) {
        S* out = (j & 1) ? Y : X;
        const S* e1 = tree + (int64_t)(p.rt.off[0] + k) * p.rec;
        bool ok;
        typename E::T kappa;
        combine<E, false>(e, L, n, e1, cur + 2 * nn, cur + 3 * nn + n, cur, out, out + nn, out + 2 * nn,
                          out + 3 * nn, out + 3 * nn + n, ok, kappa);
        ok_all = ok_all && ok;
        if (!(kappa <= kmax)) kmax = kappa;
        cur = out;
        E::sync();
    }
    fb_flag<E::NT>(p, ok_all, kmax, b, status, 4);
}

// phase 1: workgroups 0 .. batch-1 sweep the tails, the others aggregate chunks
template <typename S, class E>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_chunk_up(Plan p, S* ws, int32_t* status) {
    static_assert(!E::BIG, "wavefront engine only");
    __shared__ Lds<E> L;
    const int64_t t = blockIdx.x;
    if (t < p.batch) {
        tail_task<S, E>(L, p, ws, status, t);
    } else {
        const int64_t u = t - p.batch;
        chunk_agg_task<S, E>(L, p, ws, status, u / p.nchunk, (int)(u % p.nchunk));
    }
}

// phase 2: complete suffixes at the chunk starts, one task unit per instance.
// LW > 0 (p.leafv, chunk length 1: every chunk is a leaf): through the
// leaves' rank-m factors (leaf_combine, V' in LW row blocks)
template <typename S, class E, int LW>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_chunk_mid(Plan p, S* ws, int32_t* status) {
    static_assert(!E::BIG, "wavefront engine only");
    __shared__ Lds<E> L;
    const int64_t b = blockIdx.x;
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    bool ok_all = true;
    typename E::T kmax = 0;
    typename E::T pcar = 0;
    for (int c = p.nchunk - 1; c >= 0; --c) {
        const S* node = chunk_agg(p, tree, c);
        const S* s2 = suf + (int64_t)suffix_id(p.rt, 0, chunk_end(p, c)) * p.srec;
        S* out = suf + (int64_t)suffix_id(p.rt, 0, c * p.chunk) * p.srec;
        bool ok;
        typename E::T kappa;
        const S* first = c == p.nchunk - 1 ? s2 : (const S*)nullptr;
        if constexpr (LW > 0)
            leaf_combine<E, LW>(e, L, n, p.m, node, ws + b * p.stride + p.o_V + (int64_t)c * p.m * n, first, s2 + nn,
                                out, out + nn, ok, kappa, &pcar);
        else
            combine<E, true, sizeof(typename E::T) == 4>(e, L, n, node, first, s2 + nn, (const S*)nullptr, (S*)nullptr,
                                                         (S*)nullptr, out, (S*)nullptr, out + nn, ok, kappa, &pcar);
        ok_all = ok_all && ok;
        if (!(kappa <= kmax)) kmax = kappa;
        E::sync();
    }
    fb_flag<E::NT>(p, ok_all, kmax, b, status, 4);
}

// Chunk length 1 with the leaves built in the sweep (p.fuse_elem): the
// whole reverse scan of an instance in one task unit, from the terminal
// element (P_N = Q_N, p_N = q_N, read from the inputs) back to stage 0, each
// step leaf_elem_combine.  A factorization of R_k that fails or exceeds the
// condition threshold marks the instance as the element kernel would (bit 2
// without the fallback), a combine as the sweep would (bit 4).
template <typename S, class E, int LW>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_chunk_mid_elem(Plan p, In<S> in, S* ws,
                                                                                  int32_t* status) {
    static_assert(!E::BIG && LW > 0, "wavefront engine, leaf form");
    __shared__ Lds<E> L;
    const int64_t b = blockIdx.x;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, nn = n * n;
    const Ptr<S> P(p, in);
    S* suf = ws + b * p.stride + p.o_suf;
    {
        S* out = suf + (int64_t)suffix_id(p.rt, 0, N) * p.srec;
        coop_copy<E::NT>(out, P.Q(b, N), nn);
        coop_copy<E::NT>(out + nn, P.q(b, N), n);
    }
    bool okc_all = true, okR_all = true;
    typename E::T kc_max = 0, kR_max = 0;
    typename E::T pcar = 0;
    for (int k = N - 1; k >= 0; --k) {
        S* out = suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
        bool okc, okR;
        typename E::T kc, kR;
        leaf_elem_combine<E, LW>(e, L, p, P, b, k, k == N - 1 ? P.Q(b, N) : (const S*)nullptr, P.q(b, N), out,
                                 out + nn, okc, kc, okR, kR, &pcar);
        okc_all = okc_all && okc;
        okR_all = okR_all && okR;
        if (!(kc <= kc_max)) kc_max = kc;
        if (!(kR <= kR_max)) kR_max = kR;
        E::sync();
    }
    fb_flag<E::NT>(p, okR_all, kR_max, b, status, 2);
    fb_flag<E::NT>(p, okc_all, kc_max, b, status, 4);
}

// phase 3: the other leaves of every chunk, one task unit per chunk (LW > 0:
// through their rank-m factors, as in phase 2)
template <typename S, class E, int LW>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_chunk_down(Plan p, S* ws, int32_t* status) {
    static_assert(!E::BIG, "wavefront engine only");
    __shared__ Lds<E> L;
    const int64_t b = blockIdx.x / p.nchunk;
    const int c = (int)(blockIdx.x % p.nchunk);
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    const int c0 = c * p.chunk, c1 = chunk_end(p, c);
    bool ok_all = true;
    typename E::T kmax = 0;
    typename E::T pcar = 0;
    for (int k = c1 - 1; k > c0; --k) {
        const S* node = tree + (int64_t)(p.rt.off[0] + k) * p.rec;
        const S* s2 = suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
        S* out = suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
        bool ok;
        typename E::T kappa;
        const S* first = k == c1 - 1 ? s2 : (const S*)nullptr;
        if constexpr (LW > 0)
            leaf_combine<E, LW>(e, L, n, p.m, node, ws + b * p.stride + p.o_V + (int64_t)k * p.m * n, first, s2 + nn,
                                out, out + nn, ok, kappa, &pcar);
        else
            combine<E, true, sizeof(typename E::T) == 4>(e, L, n, node, first, s2 + nn, (const S*)nullptr, (S*)nullptr,
                                                         (S*)nullptr, out, (S*)nullptr, out + nn, ok, kappa, &pcar);
        ok_all = ok_all && ok;
        if (!(kappa <= kmax)) kmax = kappa;
        E::sync();
    }
    fb_flag<E::NT>(p, ok_all, kmax, b, status, 4);
}

// ---------------------------------------------------------------------------
// eq. (lqr) per stage, from the value function P_{k+1}, p_{k+1}:
//   G = R + B'P'B = R + (P'B)'B,  H = M' + (P'B)'A,  h = B'(p' + P'c) + r,
//   G = L_G L_G',  K = -G^{-1}H,  k = -G^{-1}h,
// then eq. (controlled_dynamics): Abar = A + B K, bbar = B k + c, written as
// the leaf of the forward tree.  Stores K, k and L_G (reused by refinement).
// ---------------------------------------------------------------------------
template <typename S, class E, int MB, bool KEEP_B = false>
__device__ __forceinline__ void policy_task(Lds<E>& L, const Plan& p, const In<S>& in, S* ws, int32_t* status,
                            int64_t task) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = task / N;
    const int k = (int)(task % N);
    const Ptr<S> P(p, in);
    S* inst = ws + b * p.stride;
    const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
    typename E::Tile t, tG, tH, tA;
    // the stage inputs go to registers first: their global latency overlaps
    // the products below (the wave barriers keep later loads from moving up)
    e.load(tA, P.A(b, k), n, n, n);
    e.load(tG, P.R(b, k), m, m, m);
    e.template load<true>(tH, P.M(b, k), m, n, m);        // M'
    // KEEP_B (the policy kernel, m <= 16): B (n x m) is read only in the
    // first MB column blocks, and the lane's part of them stays in registers
    // for both of its stagings below (no second global read); otherwise the
    // slot copy reads it each time
    T tb[E::TS][KEEP_B ? MB : 1];
    if constexpr (KEEP_B) {
        const S* Bg = P.B(b, k);
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int c = 0; c < MB; ++c)
                tb[a][c] = (e.row(a) < n && e.col(c) < m) ? T(Bg[e.row(a) * m + e.col(c)]) : T(0);
    }
    auto stage_b = [&]() {
        if constexpr (KEEP_B) {
#pragma unroll
            for (int a = 0; a < E::TS; ++a)
#pragma unroll
                for (int c = 0; c < MB; ++c) L.sX[e.row(a) * E::LD + e.col(c)] = tb[a][c];
        } else {
            stage(e, L.sX, P.B(b, k), n, m, m);
        }
    };
    stage(e, L.sA, Pn, n, n, n);                          // sA = P'
    stage_b();                                            // sX = B (first MB column blocks)
    wg_sync();
    const T v = e.template matvec<false>(L.sA, L.vb, e.vload(P.c(b, k), n), n, n) + e.vload(Pn + nn, n);
    e.zero(t);
    e.template gemm<false, false, false, false, E::TS, MB>(t, L.sA, L.sX, n);       // P'B
    const T h = e.template matvec<true>(L.sX, L.vb, v, n, m) + e.vload(P.r(b, k), m);
    wg_sync();
    e.to_lds(t, L.sA);                                    // sA = P'B
    wg_sync();
    e.template gemm<true, false, true, false, MB, MB>(tG, L.sA, L.sX, n); // R + (P'B)'B (lower)
    wg_sync();
    e.to_lds(tA, L.sX);                                   // sX = A
    wg_sync();
    e.template gemm<true, false, false, false, MB, E::TS>(tH, L.sA, L.sX, n);       // M' + (P'B)'A
    T dmin, dmax, nov[1];
    T dlA;
    const bool ok = e.template chol<0, MB>(tG, m, L.cb, dlA, nov, dmin, dmax);
    fb_flag<E::NT>(p, ok, cond_est(dmin, dmax), b, status, 2);
    e.to_lds(tG, L.sA);                                   // sA = L_G
    wg_sync();
    typename E::Tile KK[1];
#pragma unroll
    for (int a = 0; a < E::TS; ++a)
#pragma unroll
        for (int c = 0; c < E::TS; ++c) KK[0][a][c] = tH[a][c];
    T hv[1] = {h};
    e.template trsm<true, 1, 1, MB>(L.sA, dlA, m, KK, hv, L.rb);
    e.template trsm<false, 1, 1, MB>(L.sA, dlA, m, KK, hv, L.rb);
    negate<E>(KK[0]);
    hv[0] = -hv[0];
    e.store(KK[0], inst + p.o_K + (int64_t)k * m * n, m, n, n);
    e.vstore(inst + p.o_kff + (int64_t)k * m, m, hv[0]);
    e.store(tG, inst + p.o_LG + (int64_t)k * m * m, m, m, m);
    // closed loop: Abar = A + B K, bbar = B k + c
    e.to_lds(KK[0], L.sA);                                // sA = K (m x n)
    stage_b();                                            // sX = B
    wg_sync();
    e.template gemm<false, false>(tA, L.sX, L.sA, m);     // A + B K
    S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
    e.store(tA, leaf, n, n, n);
    const T bb = e.template matvec<false>(L.sX, L.vb, hv[0], m, n) + e.vload(P.c(b, k), n);
    e.vstore(leaf + nn, n, bb);
}

template <typename S, class E, int MB>
__global__ __launch_bounds__(E::NT, combine_min_waves<E>()) void k_policy(Plan p, In<S> in, S* ws, int32_t* status) {
    __shared__ Lds<E> L;
    auto body = [&](int64_t t) {
        if constexpr (E::BIG) big_policy_task<S, E>(L, p, in, ws, status, t);
        else policy_task<S, E, MB, (MB <= 2)>(L, p, in, ws, status, t);
    };
    LQR_TASKS(E, p.batch * p.N, body);
}

// ---------------------------------------------------------------------------
// forward tree up-sweep: node (l+1, i) = later (2i+1) after earlier (2i):
//   M = M_r M_l,  v = M_r v_l + v_r   (apply the earlier map first)
// VEC: only the vector part (matrices kept from the first solve).
// ---------------------------------------------------------------------------
template <typename S, class E, bool VEC, class LT>
__device__ __forceinline__ void fup_body(LT& L, Plan p, S* ws, int lvl, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const int cout = p.ft.cnt[lvl + 1], cin = p.ft.cnt[lvl];
    const int64_t b = tid / cout;
    const int i = tid % cout;
    LQR_GATE(p, b);
    S* base = ws + b * p.stride + p.o_ftree;
    const S* l = base + (int64_t)(p.ft.off[lvl] + 2 * i) * p.frec;
    S* out = base + (int64_t)(p.ft.off[lvl + 1] + i) * p.frec;
    if (2 * i + 1 >= cin) {
        if (VEC) coop_copy<E::NT>(out + nn, l + nn, n);
        else coop_copy<E::NT>(out, l, p.frec);
        return;
    }
    const S* r = l + p.frec;
    if constexpr (VEC) {
        const T v = e.template gmv<false>(r, n, n, n, e.vload(l + nn, n), L.vb[0]) + e.vload(r + nn, n);
        e.vstore(out + nn, n, v);
    } else if constexpr (E::BIG) {
        big_fup_task<S, E>(L, l, r, out, n);
    } else {
        stage(e, L.sA, r, n, n, n);                           // M_r
        stage(e, L.sX, l, n, n, n);                           // M_l
        wg_sync();
        const T v = e.template matvec<false>(L.sA, L.vb, e.vload(l + nn, n), n, n) + e.vload(r + nn, n);
        typename E::Tile t;
        e.zero(t);
        e.template gemm<false, false>(t, L.sA, L.sX, n);
        e.store(t, out, n, n, n);
        e.vstore(out + nn, n, v);
    }
}

template <typename S, class E, bool VEC>
__global__ __launch_bounds__(E::NT) void k_fup(Plan p, S* ws, int lvl) {
    __shared__ typename std::conditional<VEC, VecLds<E>, Lds<E>>::type L;
    fup_body<S, E, VEC>(L, p, ws, lvl, (int64_t)blockIdx.x);
}

// forward tree down-sweep root: start state of the whole horizon
template <typename S>
__device__ __forceinline__ void froot_body(Plan p, S* ws, const S* x0, int64_t x0_stride, int64_t tid) {
    const int64_t b = tid;
    LQR_GATE(p, b);
    const int root = p.ft.off[p.ft.nlev - 1];
    coop_copy<64>(ws + b * p.stride + p.o_xs + (int64_t)root * p.n, x0 + b * x0_stride, p.n);
}

template <typename S>
__global__ __launch_bounds__(64) void k_froot(Plan p, S* ws, const S* x0, int64_t x0_stride) {
    froot_body<S>(p, ws, x0, x0_stride, (int64_t)blockIdx.x);
}

// node (l, j): even j starts where its parent starts; odd j starts after its
// left sibling:  xs = M_{j-1} xs(parent) + v_{j-1}
template <typename S, class E, class LT>
__device__ __forceinline__ void fdown_body(LT& L, Plan p, S* ws, int lvl, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int n = p.n, nn = n * n;
    const int cnt = p.ft.cnt[lvl];
    const int64_t b = tid / cnt;
    const int j = tid % cnt;
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    const S* par = inst + p.o_xs + (int64_t)(p.ft.off[lvl + 1] + j / 2) * n;
    S* out = inst + p.o_xs + (int64_t)(p.ft.off[lvl] + j) * n;
    if ((j & 1) == 0) {
        coop_copy<E::NT>(out, par, n);
        return;
    }
    const S* sib = inst + p.o_ftree + (int64_t)(p.ft.off[lvl] + j - 1) * p.frec;
    const T x = e.template gmv<false>(sib, n, n, n, e.vload(par, n), L.vb[0]) + e.vload(sib + nn, n);
    e.vstore(out, n, x);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_fdown(Plan p, S* ws, int lvl) {
    __shared__ VecLds<E> L;
    fdown_body<S, E>(L, p, ws, lvl, (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// u_k = K_k x_k + k_k,  lambda_k = P_k x_k + p_k  (Sec. II-C); x_N from the
// last leaf map.  ADD: the refinement's correction is added to the outputs.
// ---------------------------------------------------------------------------
template <typename S, class E, bool ADD, class LT>
__device__ __forceinline__ void recover_body(LT& L, Plan p, S* ws, Out<S> out, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = tid / (N + 1);
    const int k = tid % (N + 1);
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    T x;
    if (k < N) {
        x = e.vload(inst + p.o_xs + (int64_t)k * n, n);
    } else {
        const S* leaf = inst + p.o_ftree + (int64_t)(N - 1) * p.frec;
        x = e.template gmv<false>(leaf, n, n, n, e.vload(inst + p.o_xs + (int64_t)(N - 1) * n, n), L.vb[1]) +
            e.vload(leaf + nn, n);
    }
    const S* Pk = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
    const bool hasu = k < N;
    const S* pvec = ADD ? inst + p.o_pp + (int64_t)k * n : Pk + nn;
    const T lam = e.template gmv<false>(Pk, n, n, n, x, L.vb[0]) + e.vload(pvec, n);
    T u = T(0);
    if (hasu) {
        const S* kf = ADD ? inst + p.o_kffp + (int64_t)k * m : inst + p.o_kff + (int64_t)k * m;
        u = e.template gmv<false>(inst + p.o_K + (int64_t)k * m * n, m, n, n, x, L.vb[1]) + e.vload(kf, m);
    }
    S* xo = out.x + (b * (N + 1) + k) * n;
    S* lo = out.lam + (b * (N + 1) + k) * n;
    S* uo = out.u + (b * N + k) * m;
    bool fin = true;
    if (e.lg < n) {
        const T xv = ADD ? T(xo[e.lg]) + x : x;
        const T lv = ADD ? T(lo[e.lg]) + lam : lam;
        xo[e.lg] = S(xv);
        lo[e.lg] = S(lv);
        fin = finite_(xv) && finite_(lv);
    }
    if (hasu && e.lg < m) {
        const T uv = ADD ? T(uo[e.lg]) + u : u;
        uo[e.lg] = S(uv);
        fin = fin && finite_(uv);
    }
    if (!E::all(fin)) set_status<E::NT>(out.status, b, 1);
}

template <typename S, class E, bool ADD>
__global__ __launch_bounds__(E::NT) void k_recover(Plan p, S* ws, Out<S> out) {
    __shared__ VecLds<E> L;
    recover_body<S, E, ADD>(L, p, ws, out, (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// FP64 KKT residual (stationarity of the Lagrangian of Sec. II-B plus the
// constraints), one task per (instance, stage):
//   r_init = x_0 - x0
//   r_dyn[k+1] = A x_k + B u_k + c - x_{k+1}
//   r_x[k] = Q x_k + M u_k + q + A' lam_{k+1} - lam_k   (r_x[N] = Q x_N + q - lam_N)
//   r_u[k] = M' x_k + R u_k + r + B' lam_{k+1}
// Writes the partial sums of squares (residual, right-hand side) and, when
// CORR, the correction data c' = r_dyn, q' = r_x, r' = r_u, x0' = -r_init.
// ---------------------------------------------------------------------------
template <typename S, class E, bool CORR>
__device__ __forceinline__ void resid_body(ResidLds<E>& RL, Plan p, In<S> in, const S* xs_, const S* us_, const S* ls_,
                                              S* ws, double* dws, int64_t tid) {
    static_assert(sizeof(typename E::T) == 8, "residual runs in FP64");
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m;
    const int64_t b = tid / (N + 1);
    const int k = tid % (N + 1);
    LQR_GATE(p, b);
    const Ptr<S> P(p, in);
    const S* xk = xs_ + (b * (N + 1) + k) * n;
    const S* lk = ls_ + (b * (N + 1) + k) * n;
    const double x = e.vload(xk, n), lam = e.vload(lk, n);
    double rr = 0.0, bb = 0.0;
    S* inst = ws + b * p.stride;
    // Q x + q - lam (+ M u + A' lam1 for k < N); products read straight from
    // global memory, with x, u, lam1 staged together so that the loads of
    // all the stage's matrices are in flight at once
    double qv = e.vload(P.q(b, k), n);
    e.stage_vec(RL.vb[0], x);
    if (k < N) {
        e.stage_vec(RL.vb[1], e.vload(us_ + (b * N + k) * m, m));
        e.stage_vec(RL.vb[2], e.vload(lk + n, n));
    }
    double rx = e.template gmv_v<false>(P.Q(b, k), n, n, n, RL.vb[0]) + qv - lam;
    bb += qv * qv;
    if (k < N) {
        const double x1 = e.vload(xk + n, n);
        double rd = e.template gmv_v<false>(P.A(b, k), n, n, n, RL.vb[0]);
        rx += e.template gmv_v<true>(P.A(b, k), n, n, n, RL.vb[2]);
        rd += e.template gmv_v<false>(P.B(b, k), n, m, m, RL.vb[1]);
        double ru = e.template gmv_v<true>(P.B(b, k), n, m, m, RL.vb[2]);
        rx += e.template gmv_v<false>(P.M(b, k), n, m, m, RL.vb[1]);
        ru += e.template gmv_v<true>(P.M(b, k), n, m, m, RL.vb[0]);
        const double cv = e.vload(P.c(b, k), n), rv = e.vload(P.r(b, k), m);
        ru += e.template gmv_v<false>(P.R(b, k), m, m, m, RL.vb[1]) + rv;
        rd += cv - x1;
        bb += cv * cv + rv * rv;
        rr += (e.lg < n ? rd * rd : 0.0) + (e.lg < m ? ru * ru : 0.0);
        if (CORR) {
            e.vstore(inst + p.o_cp + (int64_t)k * n, n, rd);
            e.vstore(inst + p.o_rp + (int64_t)k * m, m, ru);
        }
    }
    rr += e.lg < n ? rx * rx : 0.0;
    if (CORR) e.vstore(inst + p.o_qp + (int64_t)k * n, n, rx);
    if (k == 0) {
        const double x0v = e.vload(P.x0(b), n);
        const double ri = x - x0v;
        rr += e.lg < n ? ri * ri : 0.0;
        bb += x0v * x0v;
        if (CORR) e.vstore(inst + p.o_x0p, n, -ri);
    }
    rr = E::sum(rr);
    bb = E::sum(bb);
    if (unit_tid<E::NT>() == 0) {
        dws[b * p.dstride + 2 * k] = rr;
        dws[b * p.dstride + 2 * k + 1] = bb;
    }
}

template <typename S, class E, bool CORR>
__global__ __launch_bounds__(E::NT) void k_resid(Plan p, In<S> in, const S* xs_, const S* us_, const S* ls_,
                                              S* ws, double* dws) {
    __shared__ ResidLds<E> RL;
    resid_body<S, E, CORR>(RL, p, in, xs_, us_, ls_, ws, dws, (int64_t)blockIdx.x);
}

// rel[b] = ||r|| / ||(x0, c, q, r)||; with active_out, also mark the
// instances still above tol for another refinement sweep (never one marked
// for the FP64 redo: its FP32 factors are not usable).
template <typename D>
__global__ void k_resid_reduce(Plan p, const D* dws, D* rel, int32_t* active_out, D tol, const int32_t* status) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= p.batch) return;
    LQR_GATE(p, b);
    D rr = 0.0, bb = 0.0;
    for (int k = 0; k <= p.N; ++k) {
        rr += dws[b * p.dstride + 2 * k];
        bb += dws[b * p.dstride + 2 * k + 1];
    }
    const D r = bb > 0.0 ? __builtin_sqrt(rr) / __builtin_sqrt(bb) : __builtin_sqrt(rr);
    rel[b] = r;
    if (active_out) active_out[b] = !(r <= tol) && !(status[b] & 8);
}

// active[b] = status bit BIT of instance b is set (bit 8: marked for the
// FP64 redo; gates the residual pass that follows the redo)
template <int BIT>
__global__ void k_mark_status(const int32_t* status, int32_t* active, int64_t batch) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) active[b] = (status[b] & BIT) != 0;
}

// ---------------------------------------------------------------------------
// Refinement: correction data (x0', c', q', r') solved with the factors of
// the first solve.  With the policy fixed, the gradient recursion of eq. (lqr)
// is affine:  p'_k = Abar_k' p'_{k+1} + d_k,
//   d_k = q'_k + K_k' r'_k + Abar_k' P_{k+1} c'_k,
// a backward scan whose segment matrices are the transposes of the forward
// tree's products Abar_e ... Abar_s.
// ---------------------------------------------------------------------------
template <typename S, class E, class LT>
__device__ __forceinline__ void ref_d_body(LT& L, Plan p, S* ws, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m;
    const int64_t b = tid / N;
    const int k = tid % N;
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
    const T t = e.template gmv<false>(Pn, n, n, n, e.vload(inst + p.o_cp + (int64_t)k * n, n), L.vb[0]);
    T d = e.template gmv<true>(inst + p.o_ftree + (int64_t)k * p.frec, n, n, n, t, L.vb[1]);   // Abar_k' t
    d += e.template gmv<true>(inst + p.o_K + (int64_t)k * m * n, m, n, n,
                              e.vload(inst + p.o_rp + (int64_t)k * m, m), L.vb[0]);
    d += e.vload(inst + p.o_qp + (int64_t)k * n, n);
    e.vstore(inst + p.o_w + (int64_t)k * n, n, d);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_ref_d(Plan p, S* ws) {
    __shared__ VecLds<E> L;
    ref_d_body<S, E>(L, p, ws, (int64_t)blockIdx.x);
}

// backward up-sweep: w(l+1, i) = M(l, 2i)' w(l, 2i+1) + w(l, 2i)
template <typename S, class E, class LT>
__device__ __forceinline__ void bvec_up_body(LT& L, Plan p, S* ws, int lvl, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int n = p.n;
    const int cout = p.ft.cnt[lvl + 1], cin = p.ft.cnt[lvl];
    const int64_t b = tid / cout;
    const int i = tid % cout;
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    const S* wl = inst + p.o_w + (int64_t)(p.ft.off[lvl] + 2 * i) * n;
    S* wo = inst + p.o_w + (int64_t)(p.ft.off[lvl + 1] + i) * n;
    if (2 * i + 1 >= cin) {
        coop_copy<E::NT>(wo, wl, n);
        return;
    }
    const T w = e.template gmv<true>(inst + p.o_ftree + (int64_t)(p.ft.off[lvl] + 2 * i) * p.frec, n, n, n,
                                     e.vload(wl + n, n), L.vb[0]) + e.vload(wl, n);
    e.vstore(wo, n, w);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_bvec_up(Plan p, S* ws, int lvl) {
    __shared__ VecLds<E> L;
    bvec_up_body<S, E>(L, p, ws, lvl, (int64_t)blockIdx.x);
}

template <typename S>
__device__ __forceinline__ void broot_body(Plan p, S* ws, int64_t tid) {
    const int64_t b = tid;
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    const int root = p.ft.off[p.ft.nlev - 1];
    coop_copy<64>(inst + p.o_pend + (int64_t)root * p.n, inst + p.o_qp + (int64_t)p.N * p.n, p.n);
    coop_copy<64>(inst + p.o_pp + (int64_t)p.N * p.n, inst + p.o_qp + (int64_t)p.N * p.n, p.n);
}

template <typename S>
__global__ __launch_bounds__(64) void k_broot(Plan p, S* ws) {
    broot_body<S>(p, ws, (int64_t)blockIdx.x);
}

// backward down-sweep: pend = gradient right after the node's last stage.
//   odd j (right child): pend(parent);  even j: M(l, j+1)' pend(parent) + w(l, j+1)
template <typename S, class E, class LT>
__device__ __forceinline__ void bvec_down_body(LT& L, Plan p, S* ws, int lvl, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int n = p.n;
    const int cnt = p.ft.cnt[lvl];
    const int64_t b = tid / cnt;
    const int j = tid % cnt;
    LQR_GATE(p, b);
    S* inst = ws + b * p.stride;
    const S* par = inst + p.o_pend + (int64_t)(p.ft.off[lvl + 1] + j / 2) * n;
    S* out = inst + p.o_pend + (int64_t)(p.ft.off[lvl] + j) * n;
    if ((j & 1) || j + 1 >= cnt) {
        coop_copy<E::NT>(out, par, n);
        return;
    }
    const T v = e.template gmv<true>(inst + p.o_ftree + (int64_t)(p.ft.off[lvl] + j + 1) * p.frec, n, n, n,
                                     e.vload(par, n), L.vb[0]) +
                e.vload(inst + p.o_w + (int64_t)(p.ft.off[lvl] + j + 1) * n, n);
    e.vstore(out, n, v);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_bvec_down(Plan p, S* ws, int lvl) {
    __shared__ VecLds<E> L;
    bvec_down_body<S, E>(L, p, ws, lvl, (int64_t)blockIdx.x);
}

// v <- L^{-1} v (FWD) or L^{-T} v, L (m x m, lower, row-major) in global
// memory, v a lane vector: the pivot comes from its lane by a cross-lane
// read, every other lane updates its element (no LDS).  The steps go in
// groups of 8 whose entries of L (the lane's row or column and the
// diagonal) are loaded before the group's first step, so the dependent
// chain waits on one load per group instead of one per step.
template <bool FWD, class E, typename S>
__device__ __forceinline__ typename E::T lane_trsv(const E& e, const S* Lm, int m, typename E::T v) {
    using T = typename E::T;
    constexpr int U = 8;
    const int ng = (m + U - 1) / U;
#pragma unroll 1
    for (int gi = 0; gi < ng; ++gi) {
        const int k0 = FWD ? gi * U : (ng - 1 - gi) * U;
        T lr[U], dg[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            dg[u] = k < m ? T(Lm[k * m + k]) : T(1);
            lr[u] = (k < m && e.lg < m) ? T(FWD ? Lm[e.lg * m + k] : Lm[k * m + e.lg]) : T(0);
        }
#pragma unroll
        for (int us = 0; us < U; ++us) {
            const int u = FWD ? us : U - 1 - us;
            const int k = k0 + u;
            if (k >= m) continue;
            const T yk = __shfl(v, k, 64) / dg[u];
            if (e.lg == k) v = yk;
            else if (FWD ? (e.lg > k && e.lg < m) : (e.lg < k)) v = fma_(-lr[u], yk, v);
        }
    }
    return v;
}

// kff'_k = -G^{-1} h'_k,  h'_k = B'(p'_{k+1} + P_{k+1} c'_k) + r'_k;
// p'_k = Abar' p'_{k+1} + d_k;  new forward leaf vector B kff' + c'.
template <typename S, class E, class LT>
__device__ __forceinline__ void ref_kff_body(LT& L, Plan p, In<S> in, S* ws, int64_t tid) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = tid / N;
    const int k = tid % N;
    LQR_GATE(p, b);
    if constexpr (E::BIG) {
        big_ref_kff<S, E>(L, p, in, ws, b, k);
        return;
    } else {
    const Ptr<S> P(p, in);
    S* inst = ws + b * p.stride;
    const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
    const S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
    const T pn = e.vload(inst + p.o_pend + (int64_t)k * n, n);     // p'_{k+1}
    const T cpv = e.vload(inst + p.o_cp + (int64_t)k * n, n);
    const T v = pn + e.template gmv<false>(Pn, n, n, n, cpv, L.vb[0]);
    const T pk = e.template gmv<true>(leaf, n, n, n, pn, L.vb[1]) + e.vload(inst + p.o_w + (int64_t)k * n, n);
    e.vstore(inst + p.o_pp + (int64_t)k * n, n, pk);
    T h = e.template gmv<true>(P.B(b, k), n, m, m, v, L.vb[0]) + e.vload(inst + p.o_rp + (int64_t)k * m, m);
    const S* LG = inst + p.o_LG + (int64_t)k * m * m;
    h = lane_trsv<true>(e, LG, m, h);                      // L_G^{-1} h
    h = lane_trsv<false>(e, LG, m, h);                     // L_G^{-T} ...
    const T kf = -h;
    e.vstore(inst + p.o_kffp + (int64_t)k * m, m, kf);
    const T bb = e.template gmv<false>(P.B(b, k), n, m, m, kf, L.vb[1]) + cpv;
    e.vstore(inst + p.o_ftree + (int64_t)k * p.frec + nn, n, bb);
    }
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_ref_kff(Plan p, In<S> in, S* ws) {
    __shared__ VecLds<E> L;
    ref_kff_body<S, E>(L, p, in, ws, (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sequential vector passes (plan.fwdseq): one task unit per instance walks
// the stages in order (the forward sweep with each product's whole matrix of
// loads in flight at once, gmv_pf WIDE, so its chain waits once per product;
// in the backward sweep only the first product, since more whole ones there
// are hoisted together past the register file) and needs only the
// closed-loop leaf maps, so the
// forward tree's map products (2n^3 per node) are never formed.  For a batch
// that fills the GPU this trades the O(log N) depth of the forward scan for
// O(N n^2) work; the autotuner weighs the two.
// ---------------------------------------------------------------------------

// v <- G_k^{-1} v with the stored policy factor (L_G, or L_G^{-1} in the
// large-block engine)
template <class E, typename S>
__device__ __forceinline__ typename E::T g_solve(const E& e, const S* LG, int m, typename E::T v,
                                                 typename E::T* vb0, typename E::T* vb1) {
    if constexpr (E::BIG) {
        const typename E::T t = e.template gmv<false>(LG, m, m, m, v, vb0);
        return e.template gmv<true>(LG, m, m, m, t, vb1);
    } else {
        v = lane_trsv<true>(e, LG, m, v);
        return lane_trsv<false>(e, LG, m, v);
    }
}

// x_0 = x0, x_{k+1} = Abar_k x_k + bbar_k (eq. (controlled_dynamics)),
// u_k = K_k x_k + k_k, lambda_k = P_k x_k + p_k.  ADD: the refinement's
// correction (p' and k' from the backward sweep) is added to the outputs.
template <typename S, class E, bool ADD, class LT, bool ALT = ADD>
__device__ __forceinline__ void fwd_seq_body(LT& L, const Plan& p, S* ws, const S* x0, const Out<S>& out, int64_t b) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    S* inst = ws + b * p.stride;
    T x = e.vload(x0, n);
    bool fin = true;
    for (int k = 0; k <= N; ++k) {
        const S* Pk = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k) * p.srec;
        const S* pv = ALT ? inst + p.o_pp + (int64_t)k * n : Pk + nn;
        // x_k staged once for its three products (P_k, K_k, Abar_k), whose
        // loads then go out together
        e.stage_vec(L.vb[0], x);
        const T lam = e.template gmv_pf<false, true>(Pk, n, n, n, L.vb[0]) + e.vload(pv, n);
        S* xo = out.x + (b * (N + 1) + k) * n;
        S* lo = out.lam + (b * (N + 1) + k) * n;
        if (e.lg < n) {
            const T xv = ADD ? T(xo[e.lg]) + x : x;
            const T lv = ADD ? T(lo[e.lg]) + lam : lam;
            xo[e.lg] = S(xv);
            lo[e.lg] = S(lv);
            fin = fin && finite_(xv) && finite_(lv);
        }
        if (k == N) break;
        const S* kf = inst + (ALT ? p.o_kffp : p.o_kff) + (int64_t)k * m;
        const T u = e.template gmv_pf<false, true>(inst + p.o_K + (int64_t)k * m * n, m, n, n, L.vb[0]) + e.vload(kf, m);
        S* uo = out.u + (b * N + k) * m;
        if (e.lg < m) {
            const T uv = ADD ? T(uo[e.lg]) + u : u;
            uo[e.lg] = S(uv);
            fin = fin && finite_(uv);
        }
        const S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
        x = e.template gmv_pf<false, true>(leaf, n, n, n, L.vb[0]) + e.vload(leaf + nn, n);
    }
    if (!E::all(fin)) set_status<E::NT>(out.status, b, 1);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_fwd_seq(Plan p, S* ws, const S* x0, Out<S> out) {
    __shared__ VecLds<E> L;
    const int64_t b = blockIdx.x;
    fwd_seq_body<S, E, false>(L, p, ws, x0 + b * p.n, out, b);
}

// Backward sweep of the gradient recursion of eq. (lqr) with the policy of
// the first solve fixed, for right-hand sides (c', q', r') read from the
// workspace's refinement area (RHS_IN false) or from the inputs (true):
//   v = p'_{k+1} + P_{k+1} c'_k,  k'_k = -G_k^{-1}(B_k' v + r'_k),
//   p'_k = Abar_k' v + K_k' r'_k + q'_k,
// storing p'_k, k'_k and the closed-loop offsets B_k k'_k + c'_k over the
// leaf vectors.
template <typename S, class E, bool RHS_IN, class LT>
__device__ __forceinline__ void bwd_seq_body(LT& L, const Plan& p, const In<S>& in, S* ws, int64_t b) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const Ptr<S> P(p, in);
    S* inst = ws + b * p.stride;
    auto qv = [&](int k) { return RHS_IN ? P.q(b, k) : (const S*)(inst + p.o_qp + (int64_t)k * n); };
    T pn = e.vload(qv(N), n);
    e.vstore(inst + p.o_pp + (int64_t)N * n, n, pn);
    for (int k = N - 1; k >= 0; --k) {
        const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
        S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
        const T cpv = e.vload(RHS_IN ? P.c(b, k) : (const S*)(inst + p.o_cp + (int64_t)k * n), n);
        const T rpv = e.vload(RHS_IN ? P.r(b, k) : (const S*)(inst + p.o_rp + (int64_t)k * m), m);
        // products grouped by the vector they need: (P_{k+1} c', K' r')
        // first, then (B' v, Abar' v), so each group's loads go out together
        e.stage_vec(L.vb[0], cpv);
        e.stage_vec(L.vb[1], rpv);
        const T v = pn + e.template gmv_pf<false, true>(Pn, n, n, n, L.vb[0]);
        const T kr = e.template gmv_pf<true>(inst + p.o_K + (int64_t)k * m * n, m, n, n, L.vb[1]);
        e.stage_vec(L.vb[0], v);
        const T h = e.template gmv_pf<true>(P.B(b, k), n, m, m, L.vb[0]) + rpv;
        pn = e.template gmv_pf<true>(leaf, n, n, n, L.vb[0]) + kr + e.vload(qv(k), n);
        e.vstore(inst + p.o_pp + (int64_t)k * n, n, pn);
        const T kf = -g_solve(e, inst + p.o_LG + (int64_t)k * m * m, m, h, L.vb[0], L.vb[1]);
        e.vstore(inst + p.o_kffp + (int64_t)k * m, m, kf);
        e.stage_vec(L.vb[1], kf);
        const T bb = e.template gmv_pf<false>(P.B(b, k), n, m, m, L.vb[1]) + cpv;
        e.vstore(leaf + nn, n, bb);
        E::sync();
    }
}

// One refinement sweep of instance b with the factors of the first solve
// (after the FP64 residual pass wrote c', q', r', x0'): the backward sweep
// above on the correction data, then the forward sweep of the correction,
// added to the outputs.
template <typename S, class E, class LT>
__device__ __forceinline__ void refine_seq_body(LT& L, const Plan& p, const In<S>& in, S* ws, const Out<S>& out,
                                                int64_t b) {
    bwd_seq_body<S, E, false>(L, p, in, ws, b);
    fwd_seq_body<S, E, true>(L, p, ws, (const S*)(ws + b * p.stride + p.o_x0p), out, b);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_refine_seq(Plan p, In<S> in, S* ws, Out<S> out) {
    __shared__ VecLds<E> L;
    const int64_t b = blockIdx.x;
    LQR_GATE(p, b);
    refine_seq_body<S, E>(L, p, in, ws, out, b);
}

// Re-solve with the cached factors: the value function, policy and
// closed-loop matrices of the last solve of these matrices stay in the
// workspace, new (x0, c, q, r) come from the inputs: the backward sweep on
// them, then the forward sweep.  O(N n^2) per instance.  Instances the last
// solve sent to the FP64 redo (status bit 8) are skipped here (their FP32
// factors are not usable; the redo launch solves them again).
template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_resolve_seq(Plan p, In<S> in, S* ws, Out<S> out) {
    __shared__ VecLds<E> L;
    const int64_t b = blockIdx.x;
    if (out.status[b] & 8) return;
    bwd_seq_body<S, E, true>(L, p, in, ws, b);
    fwd_seq_body<S, E, false, VecLds<E>, true>(L, p, ws, in.x0 + b * p.n, out, b);
}

// relative KKT residual of instance b from its per-stage partial sums
__device__ __forceinline__ double resid_of_parts(const Plan& p, const double* dws, int64_t b) {
    double rr = 0.0, bb = 0.0;
    for (int k = 0; k <= p.N; ++k) {
        rr += dws[b * p.dstride + 2 * k];
        bb += dws[b * p.dstride + 2 * k + 1];
    }
    return bb > 0.0 ? __builtin_sqrt(rr) / __builtin_sqrt(bb) : __builtin_sqrt(rr);
}

// ---------------------------------------------------------------------------
// Per-instance forms of the vector-only passes: one workgroup per instance
// walks every stage and tree node of its instance in order.  For large
// batches these replace the level-by-level launches, whose tiny O(n^2)
// tasks are bound by the workgroup launch rate.  Every vector a task leaves
// in global memory is read back only by the lane that wrote it (element lg
// by lane lg: vload/vstore/coop_copy all map element i to lane i for
// i < 64), so single-thread program order suffices between tasks; the only
// cross-lane hand-offs are the LDS ones inside the products.
// ---------------------------------------------------------------------------

// forward scan of the closed-loop maps from x0 (UPV: recompute the vector
// part of the up-sweep first) and u_k, lambda_k (ADD: added to the outputs)
template <typename S, class E, bool UPV, bool ADD, class LT>
__device__ __forceinline__ void fwd_inst_body(LT& L, const Plan& p, S* ws, const S* x0, int64_t x0_stride,
                                              const Out<S>& out, int64_t b) {
    if (UPV) {
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            for (int i = 0; i < p.ft.cnt[l + 1]; ++i) {
                fup_body<S, E, true>(L, p, ws, l, b * p.ft.cnt[l + 1] + i);
                E::sync();
            }
        }
    }
    froot_body<S>(p, ws, x0, x0_stride, b);
    E::sync();
    for (int l = p.ft.nlev - 2; l >= 0; --l) {
        for (int j = 0; j < p.ft.cnt[l]; ++j) {
            fdown_body<S, E>(L, p, ws, l, b * p.ft.cnt[l] + j);
            E::sync();
        }
    }
    for (int k = 0; k <= p.N; ++k) {
        recover_body<S, E, ADD>(L, p, ws, out, b * (p.N + 1) + k);
        E::sync();
    }
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_fwd_inst(Plan p, S* ws, const S* x0, int64_t x0_stride, Out<S> out) {
    __shared__ VecLds<E> L;
    const int64_t b = blockIdx.x;
    LQR_GATE(p, b);
    fwd_inst_body<S, E, false, false>(L, p, ws, x0, x0_stride, out, b);
}

// one whole refinement sweep of one instance (after its residual pass)
template <typename S, class E, class LT>
__device__ __forceinline__ void refine_inst_body(LT& L, const Plan& p, const In<S>& in, S* ws, const Out<S>& out,
                                                 int64_t b) {
    const int N = p.N;
    for (int k = 0; k < N; ++k) {
        ref_d_body<S, E>(L, p, ws, b * N + k);
        E::sync();
    }
    E::sync();
    for (int l = 0; l + 1 < p.ft.nlev; ++l) {
        for (int i = 0; i < p.ft.cnt[l + 1]; ++i) {
            bvec_up_body<S, E>(L, p, ws, l, b * p.ft.cnt[l + 1] + i);
            E::sync();
        }
    }
    broot_body<S>(p, ws, b);
    E::sync();
    for (int l = p.ft.nlev - 2; l >= 0; --l) {
        for (int j = 0; j < p.ft.cnt[l]; ++j) {
            bvec_down_body<S, E>(L, p, ws, l, b * p.ft.cnt[l] + j);
            E::sync();
        }
    }
    for (int k = 0; k < N; ++k) {
        ref_kff_body<S, E>(L, p, in, ws, b * N + k);
        E::sync();
    }
    E::sync();
    fwd_inst_body<S, E, true, true>(L, p, ws, (const S*)(ws + p.o_x0p), p.stride, out, b);
}

template <typename S, class E>
__global__ __launch_bounds__(E::NT) void k_refine_inst(Plan p, In<S> in, S* ws, Out<S> out) {
    __shared__ VecLds<E> L;
    const int64_t b = blockIdx.x;
    LQR_GATE(p, b);
    refine_inst_body<S, E>(L, p, in, ws, out, b);
}

// FP64 residual of one instance, all stages, reduced in place:
// rel[b] = ||r|| / ||(x0, c, q, r)|| (and active_out[b] = rel > tol for an
// instance not marked for the FP64 redo)
template <typename S, class E, bool CORR>
__device__ __forceinline__ double resid_inst_body(ResidLds<E>& RL, const Plan& p, const In<S>& in, const S* xs_,
                                                  const S* us_, const S* ls_, S* ws, double* dws, double* rel,
                                                  int32_t* active_out, double tol, const int32_t* status, int64_t b) {
    double res = 0.0;   // returned in the task unit's thread 0
    for (int k = 0; k <= p.N; ++k) {
        resid_body<S, E, CORR>(RL, p, in, xs_, us_, ls_, ws, dws, b * (p.N + 1) + k);
        E::sync();
    }
    if (unit_tid<E::NT>() == 0) {   // the partial sums were written by this lane
        const double r = resid_of_parts(p, dws, b);
        if (rel) rel[b] = r;
        if (active_out) active_out[b] = !(r <= tol) && !(status[b] & 8);
        res = r;
    }
    return res;
}

template <typename S, class E, bool CORR>
__global__ __launch_bounds__(E::NT) void k_resid_inst(Plan p, In<S> in, const S* xs_, const S* us_, const S* ls_,
                                                   S* ws, double* dws, double* rel, int32_t* active_out,
                                                   double tol, const int32_t* status) {
    __shared__ ResidLds<E> RL;
    const int64_t b = blockIdx.x;
    LQR_GATE(p, b);
    resid_inst_body<S, E, CORR>(RL, p, in, xs_, us_, ls_, ws, dws, rel, active_out, tol, status, b);
}

// ---------------------------------------------------------------------------
// Plain baseline: the sequential Riccati recursion of eq. (lqr), forward pass
// and costates, one group per instance.  Inputs and outputs are of type S;
// the intermediates (P_k, p_k in the suffix area indexed by stage, K_k, k_k)
// live in `inst` of type W (W = S for the baseline, double for the FP64
// redo of an FP32 instance).
// ---------------------------------------------------------------------------
template <typename S, typename W, class E, int MB>
__device__ __forceinline__ void plain_body(Lds3<E>& L, const Plan& p, const In<S>& in, const Out<S>& out, W* inst,
                                           int64_t b) {
    using T = typename E::T;
    const E e(unit_tid<E::NT>());
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const Ptr<S> P(p, in);
    W* Pst = inst + p.o_suf;                               // P_k, p_k at k * srec
    typename E::Tile t, tPB, tG, tH, tHc, tPA;
    e.load(t, P.Q(b, N), n, n, n);
    to_lds_sym(e, t, L.sP);
    e.store_sym(t, Pst + (int64_t)N * p.srec, n);
    T pn = e.vload(P.q(b, N), n);
    e.vstore(Pst + (int64_t)N * p.srec + nn, n, pn);
    bool ok = true;
    for (int k = N - 1; k >= 0; --k) {
        wg_sync();
        stage(e, L.sX, P.B(b, k), n, m, m);               // sX = B
        wg_sync();
        const T v = e.template matvec<false>(L.sP, L.vb, e.vload(P.c(b, k), n), n, n) + pn;
        e.zero(tPB);
        e.template gemm<false, false, false, false, E::TS, MB>(tPB, L.sP, L.sX, n); // P'B
        const T h = e.template matvec<true>(L.sX, L.vb, v, n, m) + e.vload(P.r(b, k), m);
        wg_sync();
        e.to_lds(tPB, L.sA);                              // sA = P'B
        wg_sync();
        e.load(tG, P.R(b, k), m, m, m);
        e.template gemm<true, false, true, false, MB, MB>(tG, L.sA, L.sX, n);   // G (lower)
        wg_sync();
        stage(e, L.sX, P.A(b, k), n, n, n);               // sX = A
        wg_sync();
        e.template load<true>(tH, P.M(b, k), m, n, m);
        e.template gemm<true, false, false, false, MB, E::TS>(tH, L.sA, L.sX, n);   // H
        e.zero(tPA);
        e.template gemm<false, false>(tPA, L.sP, L.sX, n); // P'A
        const T pa = e.template matvec<true>(L.sX, L.vb, v, n, n);   // A'v
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int c = 0; c < E::TS; ++c) tHc[a][c] = tH[a][c];
        T dmin, dmax, nov[1];
        T dlA;
        ok = e.template chol<0, MB>(tG, m, L.cb, dlA, nov, dmin, dmax) && ok;
        e.to_lds(tG, L.sA);                               // sA = L_G
        wg_sync();
        typename E::Tile KK[1];
#pragma unroll
        for (int a = 0; a < E::TS; ++a)
#pragma unroll
            for (int c = 0; c < E::TS; ++c) KK[0][a][c] = tH[a][c];
        T hv[1] = {h};
        e.template trsm<true, 1, 1, MB>(L.sA, dlA, m, KK, hv, L.rb);
        e.template trsm<false, 1, 1, MB>(L.sA, dlA, m, KK, hv, L.rb);
        negate<E>(KK[0]);
        hv[0] = -hv[0];
        e.store(KK[0], inst + p.o_K + (int64_t)k * m * n, m, n, n);
        e.vstore(inst + p.o_kff + (int64_t)k * m, m, hv[0]);
        // P_k = Q + A'(P'A) + K'H,  p_k = q + A'v + K'h
        wg_sync();
        e.to_lds(tPA, L.sP);                              // sP = P'A
        wg_sync();
        e.load(t, P.Q(b, k), n, n, n);
        e.template gemm<true, false, true>(t, L.sX, L.sP, n);   // Q + A'(P'A) (lower)
        wg_sync();
        e.to_lds(KK[0], L.sA);                            // sA = K
        e.to_lds(tHc, L.sX);                              // sX = H
        wg_sync();
        e.template gemm<true, false, true>(t, L.sA, L.sX, m);   // + K'H (lower)
        pn = e.vload(P.q(b, k), n) + pa + e.template matvec<true>(L.sA, L.vb, h, m, n);
        wg_sync();
        to_lds_sym(e, t, L.sP);
        e.store_sym(t, Pst + (int64_t)k * p.srec, n);
        e.vstore(Pst + (int64_t)k * p.srec + nn, n, pn);
    }
    if (!ok) set_status<E::NT>(out.status, b, 2);
    // forward pass and costates
    T x = e.vload(P.x0(b), n);
    bool fin = true;
    for (int k = 0; k <= N; ++k) {
        wg_sync();
        stage(e, L.sP, Pst + (int64_t)k * p.srec, n, n, n);
        if (k < N) {
            stage(e, L.sA, inst + p.o_K + (int64_t)k * m * n, m, n, n);
            stage(e, L.sX, P.A(b, k), n, n, n);
        }
        wg_sync();
        const T lam = e.template matvec<false>(L.sP, L.vb, x, n, n) + e.vload(Pst + (int64_t)k * p.srec + nn, n);
        e.vstore(out.x + (b * (N + 1) + k) * n, n, x);
        e.vstore(out.lam + (b * (N + 1) + k) * n, n, lam);
        fin = fin && (e.lg >= n || (finite_(x) && finite_(lam)));
        if (k == N) break;
        const T u = e.template matvec<false>(L.sA, L.vb, x, n, m) + e.vload(inst + p.o_kff + (int64_t)k * m, m);
        e.vstore(out.u + (b * N + k) * m, m, u);
        fin = fin && (e.lg >= m || finite_(u));
        wg_sync();
        T xn = e.template matvec<false>(L.sX, L.vb, x, n, n) + e.vload(P.c(b, k), n);
        wg_sync();
        stage(e, L.sA, P.B(b, k), n, m, m);
        wg_sync();
        xn += e.template matvec<false>(L.sA, L.vb, u, m, n);
        x = xn;
    }
    if (!wave_all(fin)) set_status<E::NT>(out.status, b, 1);
}

template <typename S, class E, int MB>
__global__ __launch_bounds__(64) void k_plain(Plan p, In<S> in, Out<S> out, S* ws) {
    __shared__ Lds3<E> L;
    const int64_t b = blockIdx.x;
    plain_body<S, S, E, MB>(L, p, in, out, ws + b * p.stride, b);
}

// FP64 redo of the instances an FP32 solve marked (status bit 8): each is
// solved again whole by the sequential Riccati recursion of eq. (lqr) with
// FP64 arithmetic and FP64 intermediates (one FP64 slot of `rp.stride`
// doubles per workgroup), and its FP32 outputs are overwritten.  The status
// word keeps bit 8 and gets the failure bits of this solve.  `rp` is the
// plan of the redo slots (batch = the instance count of the call).
template <typename S, class E64, int MB>
__global__ __launch_bounds__(64) void k_redo(Plan rp, In<S> in, Out<S> out, double* ws64) {
    __shared__ Lds3<E64> L;
    for (int64_t b = blockIdx.x; b < rp.batch; b += gridDim.x) {
        if (!(out.status[b] & 8)) continue;   // uniform: one status word per workgroup iteration
        wg_sync();
        if (threadIdx.x == 0) out.status[b] = 8;
        plain_body<S, double, E64, MB>(L, rp, in, out, ws64 + (int64_t)blockIdx.x * rp.stride, b);
    }
}

// ---------------------------------------------------------------------------
// Fused solve (wavefront engine): one workgroup of W wavefronts runs one
// instance from its elements to its last refinement sweep (Sec. II-D
// elements, reverse scan, policy, forward scan, recovery; FP64 residual and
// refinement) in a single launch.  Each phase of the launch sequence (the
// stages of a per-stage pass, the nodes of one tree level) becomes a loop
// whose tasks are spread over the wavefronts, each wavefront with LDS slots
// of its own, and a workgroup barrier separates dependent phases.  Every
// task body is the one the launch sequence uses, in the same phase order,
// so an instance gets the bits of the launched form.
// An instance a factorization marks (status bit 8) is solved again whole by
// the FP64 redo launch that follows (k_redo).
// ---------------------------------------------------------------------------
template <class E, class E64>
struct FusedLds {
    Lds<E> m;          // matrix tasks
    VecLds<E> v;       // vector-only tasks
    ResidLds<E64> r;   // FP64 residual
};

template <class E>
constexpr int fused_waves() {
    using F = FusedLds<E, Eng<double, E::G, E::TS>>;
    constexpr int lim = E::TS <= 2 ? 8 : 4;
    constexpr int w = (int)(65536 / sizeof(F));
    return w < 1 ? 1 : (w > lim ? lim : w);
}

// The whole solve of instance b by the W wavefronts of the calling
// workgroup (F: their LDS, sh_rel: one shared double).
template <typename S, class E, class E64, int MB>
__device__ __forceinline__ void fused_body(FusedLds<E, E64>* F, double& sh_rel, const Plan& p, const In<S>& in,
                                           const Out<S>& out, S* ws, double* dws, double* rel_out,
                                           const Warm<S>& warm, int refine, int64_t b) {
    static_assert(!E::BIG && E::NT == 64, "wavefront engine only");
    constexpr int W = fused_waves<E>();
    const int wv = (int)(threadIdx.x >> 6);
    const int N = p.N, n = p.n;
    auto& Lm = F[wv].m;
    auto& Lv = F[wv].v;
    auto& Lr = F[wv].r;
    // one phase: tasks t = wv, wv + W, ... < count, then the workgroup barrier
    auto phase = [&](int count, auto&& body) {
        for (int t = wv; t < count; t += W) {
            body(t);
            E::sync();
        }
        __syncthreads();
    };
    if (threadIdx.x == 0) out.status[b] = 0;
    __syncthreads();
    // elements; reverse scan (up-sweep, root, down-sweep); policy and
    // closed-loop maps; up-sweep of the forward tree
    phase(N + 1, [&](int k) { element_task<S, E, MB>(Lm, p, in, ws, out.status, b * (N + 1) + k); });
    for (int l = 0; l + 1 < p.rt.nlev; ++l) {
        const int c = p.rt.cnt[l + 1];
        phase(c, [&](int i) { up_task<S, E>(Lm, p, ws, l, out.status, b * c + i); });
    }
    phase(1, [&](int) { root_body<S>(p, ws, b); });
    for (int l = p.rt.nlev - 2; l >= 0; --l) {
        const int c = p.rt.cnt[l] / 2;
        phase(c, [&](int j) { down_task<S, E>(Lm, p, ws, l, out.status, b * c + j); });
    }
    phase(N, [&](int k) { policy_task<S, E, MB>(Lm, p, in, ws, out.status, b * N + k); });
    for (int l = 0; l + 1 < p.ft.nlev; ++l) {
        const int c = p.ft.cnt[l + 1];
        phase(c, [&](int i) { fup_body<S, E, false>(Lm, p, ws, l, b * c + i); });
    }
    // forward down-sweep from a start state, then u_k, lambda_k (ADD: the
    // refinement's correction is added to the outputs)
    auto forward = [&](const S* x0, int64_t x0_stride, auto add) {
        constexpr bool ADD = decltype(add)::value;
        phase(1, [&](int) { froot_body<S>(p, ws, x0, x0_stride, b); });
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const int c = p.ft.cnt[l];
            phase(c, [&](int j) { fdown_body<S, E>(Lv, p, ws, l, b * c + j); });
        }
        phase(N + 1, [&](int k) { recover_body<S, E, ADD>(Lv, p, ws, out, b * (N + 1) + k); });
    };
    // FP64 residual of the current outputs (CORR: also the right-hand sides
    // of the correction); the same value in every thread
    auto residual = [&](auto corr) -> double {
        constexpr bool CORR = decltype(corr)::value;
        phase(N + 1, [&](int k) {
            resid_body<S, E64, CORR>(Lr, p, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws,
                                     b * (N + 1) + k);
        });
        if (threadIdx.x == 0) {
            const double r = resid_of_parts(p, dws, b);
            sh_rel = r;
            if (rel_out) rel_out[b] = r;
        }
        __syncthreads();
        return sh_rel;
    };
    int sweeps = refine;
    if (warm.x) {
        const int cx = (N + 1) * n, cu = N * p.m;
        for (int i = (int)threadIdx.x; i < cx; i += 64 * W) {
            if (warm.x != out.x) out.x[b * cx + i] = warm.x[b * cx + i];
            if (warm.lam != out.lam) out.lam[b * cx + i] = warm.lam[b * cx + i];
        }
        for (int i = (int)threadIdx.x; i < cu; i += 64 * W)
            if (warm.u != out.u) out.u[b * cu + i] = warm.u[b * cu + i];
        __syncthreads();
        if (sweeps < 1) sweeps = 1;
    } else {
        forward(in.x0, (int64_t)n, std::false_type{});
    }
    // refinement sweeps while the residual is above the tolerance
    bool changed = true;   // outputs changed since the last residual
    for (int sw = 0; sw < sweeps; ++sw) {
        const double r = residual(std::true_type{});
        changed = false;
        if (r <= p.refine_tol) break;
        phase(N, [&](int k) { ref_d_body<S, E>(Lv, p, ws, b * N + k); });
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const int c = p.ft.cnt[l + 1];
            phase(c, [&](int i) { bvec_up_body<S, E>(Lv, p, ws, l, b * c + i); });
        }
        phase(1, [&](int) { broot_body<S>(p, ws, b); });
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const int c = p.ft.cnt[l];
            phase(c, [&](int j) { bvec_down_body<S, E>(Lv, p, ws, l, b * c + j); });
        }
        phase(N, [&](int k) { ref_kff_body<S, E>(Lv, p, in, ws, b * N + k); });
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const int c = p.ft.cnt[l + 1];
            phase(c, [&](int i) { fup_body<S, E, true>(Lv, p, ws, l, b * c + i); });
        }
        forward((const S*)(ws + p.o_x0p), p.stride, std::true_type{});
        changed = true;
    }
    if (rel_out && changed) residual(std::false_type{});
}

template <typename S, class E, class E64, int MB>
__global__ __launch_bounds__(64 * fused_waves<E>()) void k_solve_fused(Plan p, In<S> in, Out<S> out, S* ws,
                                                                      double* dws, double* rel_out, Warm<S> warm,
                                                                      int refine) {
    __shared__ FusedLds<E, E64> F[fused_waves<E>()];
    __shared__ double sh_rel;
    fused_body<S, E, E64, MB>(F, sh_rel, p, in, out, ws, dws, rel_out, warm, refine, (int64_t)blockIdx.x);
}

// ---------------------------------------------------------------------------
// Ragged batches from a device descriptor table: persistent workgroups (one
// workspace slot each) take problems from an atomic counter and solve each
// whole (fused_body) with a plan built on the device from its sizes.  One
// launch per padded-order class; a launch skips the problems of the other
// classes.  Problems are addressed as instance 0 of a batch of one: their
// arrays are offsets into packed buffers, their status and residual words
// are at status_idx.
// ---------------------------------------------------------------------------
struct RaggedDesc {
    int32_t N, n, m, status_idx;
    int64_t in_off[9], out_off[3];
};

// padded-order class of a problem on the wavefront engine (0: none)
__host__ __device__ inline int wave_class(int n, int m) {
    const int d = n > m ? n : m;
    const int ts = (d + 7) / 8;
    return d < 1 ? 0 : ts <= 6 ? ts : ts <= 8 ? 8 : 0;
}

template <typename S>
struct RaggedArgs {
    const RaggedDesc* desc;
    int64_t count;
    const S* in;           // packed inputs
    S* out;                // packed outputs
    int32_t* status;       // [count], by status_idx
    double* rel;           // [count] by status_idx, or nullptr
    S* ws;                 // slots of slot_elems
    int64_t slot_elems;
    double* dws;           // FP64 partial sums, dslot per slot
    int64_t dslot;
    double* ws64;          // FP64 redo slots of slot64 doubles
    int64_t slot64;
    const S *warm_x, *warm_u, *warm_lam;   // packed like the outputs, or nullptr (cold)
    int32_t* counter;      // work counter of this launch (zero before it)
    int maxN, maxd;        // bounds the slots were sized for
    int refine, fallback;
    double cond_thr, refine_tol;
};

// plan of problem d (instance 0 of a batch of one); false if the problem
// is malformed or larger than the slots
template <typename S>
__device__ __forceinline__ bool ragged_plan(const RaggedArgs<S>& a, const RaggedDesc& d, Plan& p) {
    if (d.N < 1 || d.n < 1 || d.m < 1 || d.N > a.maxN || d.n > a.maxd || d.m > a.maxd) return false;
    p = Plan{};
    p.batch = 1;
    plan_records(p, d.N, d.n, d.m, false);   // the one-launch solve combines leaves in the general form
    p.cond_thr = a.cond_thr;
    p.refine_tol = a.refine_tol;
    p.fallback = a.fallback;
    return p.stride <= a.slot_elems && p.dstride + 1 <= a.dslot;
}

template <typename S>
__device__ __forceinline__ In<S> ragged_in(const RaggedArgs<S>& a, const RaggedDesc& d) {
    return In<S>{a.in + d.in_off[0], a.in + d.in_off[1], a.in + d.in_off[2], a.in + d.in_off[3], a.in + d.in_off[4],
                 a.in + d.in_off[5], a.in + d.in_off[6], a.in + d.in_off[7], a.in + d.in_off[8]};
}

// the next problem index of this workgroup's loop (same value in every thread)
__device__ __forceinline__ int64_t ragged_next(int32_t* counter, int64_t* sh) {
    __syncthreads();
    if (threadIdx.x == 0) *sh = atomicAdd(counter, 1);
    __syncthreads();
    return *sh;
}

template <typename S, class E, class E64>
__global__ __launch_bounds__(64 * fused_waves<E>()) void k_ragged_fused(RaggedArgs<S> a) {
    __shared__ FusedLds<E, E64> F[fused_waves<E>()];
    __shared__ double sh_rel;
    __shared__ int64_t sh_i;
    S* slot = a.ws + (int64_t)blockIdx.x * a.slot_elems;
    double* dslot = a.dws + (int64_t)blockIdx.x * a.dslot;
    for (int64_t i = ragged_next(a.counter, &sh_i); i < a.count; i = ragged_next(a.counter, &sh_i)) {
        const RaggedDesc d = a.desc[i];
        if (d.status_idx < 0 || d.status_idx >= a.count || wave_class(d.n, d.m) != E::TS) continue;
        Plan p;
        if (!ragged_plan(a, d, p)) continue;
        const Out<S> out{a.out + d.out_off[0], a.out + d.out_off[1], a.out + d.out_off[2], a.status + d.status_idx};
        const Warm<S> warm = a.warm_x ? Warm<S>{a.warm_x + d.out_off[0], a.warm_u + d.out_off[1],
                                                a.warm_lam + d.out_off[2]}
                                      : Warm<S>{nullptr, nullptr, nullptr};
        fused_body<S, E, E64, E::TS>(F, sh_rel, p, ragged_in(a, d), out, slot, dslot,
                                     a.rel ? a.rel + d.status_idx : nullptr, warm, a.refine, 0);
    }
}

// FP64 redo of the marked problems of one class (as k_redo), then the FP64
// residual of the new solution
template <typename S, class E64>
__global__ __launch_bounds__(64) void k_ragged_redo(RaggedArgs<S> a) {
    __shared__ Lds3<E64> L;
    __shared__ ResidLds<E64> RL;
    __shared__ int64_t sh_i;
    double* slot64 = a.ws64 + (int64_t)blockIdx.x * a.slot64;
    double* dslot = a.dws + (int64_t)blockIdx.x * a.dslot;
    for (int64_t i = ragged_next(a.counter, &sh_i); i < a.count; i = ragged_next(a.counter, &sh_i)) {
        const RaggedDesc d = a.desc[i];
        if (d.status_idx < 0 || d.status_idx >= a.count || wave_class(d.n, d.m) != E64::TS) continue;
        if (!(a.status[d.status_idx] & 8)) continue;
        Plan p;
        if (!ragged_plan(a, d, p)) continue;
        Plan r = p;
        redo_records(r);
        if (r.stride > a.slot64) continue;
        const In<S> in = ragged_in(a, d);
        const Out<S> out{a.out + d.out_off[0], a.out + d.out_off[1], a.out + d.out_off[2], a.status + d.status_idx};
        wg_sync();
        if (threadIdx.x == 0) *out.status = 8;
        plain_body<S, double, E64, E64::TS>(L, r, in, out, slot64, 0);
        wg_sync();
        if (a.rel)
            resid_inst_body<S, E64, false>(RL, p, in, out.x, out.u, out.lam, (S*)nullptr, dslot, a.rel + d.status_idx,
                                           (int32_t*)nullptr, p.refine_tol, (const int32_t*)nullptr, 0);
    }
}

// status words of the problems no class launch takes (malformed sizes,
// orders above the wavefront classes, larger than the slots): bit 16
template <typename S>
__global__ void k_ragged_check(RaggedArgs<S> a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const RaggedDesc d = a.desc[i];
    if (d.status_idx < 0 || d.status_idx >= a.count) return;
    Plan p;
    const bool ok = wave_class(d.n, d.m) != 0 && ragged_plan(a, d, p);
    a.status[d.status_idx] = ok ? 0 : 16;
    if (!ok && a.rel) a.rel[d.status_idx] = -1.0;
}

}  // namespace lqr
