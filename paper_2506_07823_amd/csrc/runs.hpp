// runs.hpp -- launch sequences of the scan, plain and residual paths.
//
// Instantiated once per padded-order class (inst.hip with LQR_TS defined) so
// the classes compile in parallel; lqr_kkt.hip dispatches to them.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "../../include/lqr_kkt.h"
#include "kernels.hpp"

namespace lqr {

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess) return fail(LQR_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int WG = 64;
// shape class of the large-block engine (orders 65..256)
constexpr int kBigTS = 32;

template <typename S, int TS>
using EngOf = typename std::conditional<TS == kBigTS, BigEng<S>, Eng<S, 8, TS>>::type;

// Row blocks of the leaves' rank-m factors for the sweeps of the chunked
// schedule (p.leafv: m <= 16 at orders 17..64, i.e. one or two blocks of a
// tile of at least three), 0: the general cheap combine
template <int TS, typename Fn>
int with_lw(const Plan& p, Fn&& fn) {
    if constexpr (TS != kBigTS && TS > 2) {
        if (p.leafv && p.m <= 8) return fn(std::integral_constant<int, 1>{});
        if (p.leafv && p.m <= 16) return fn(std::integral_constant<int, 2>{});
    }
    return fn(std::integral_constant<int, 0>{});
}

// host-side choice of the control-block count MB (see kernels.hpp): calls
// fn(std::integral_constant<int, MB>) with MB = 1, 2 or TS (0 for the
// large-block engine, which does not use it)
template <int TS, typename Fn>
int with_mb(int m, Fn&& fn) {
    if constexpr (TS == kBigTS) {
        return fn(std::integral_constant<int, 0>{});
    } else {
        const int mb = (m + 7) / 8;
        if constexpr (TS > 1) {
            if (mb <= 1) return fn(std::integral_constant<int, 1>{});
        }
        if constexpr (TS > 2) {
            if (mb <= 2) return fn(std::integral_constant<int, 2>{});
        }
        return fn(std::integral_constant<int, TS>{});
    }
}

// kernel families (diagnostic timing keys)
enum Fam {
    F_CLEAR, F_ELEM, F_UP, F_ROOT, F_DOWN, F_POLICY, F_FUP, F_FROOT, F_FDOWN, F_RECOVER, F_RESID, F_REF_D, F_BUP,
    F_BROOT, F_BDOWN, F_REF_KFF, F_FUPV, F_RECOVER_ADD, F_REDUCE, F_PLAIN, F_FWD_INST, F_REFINE_INST, F_WARM, F_PACK,
    F_FUSED, F_TAIL, F_TROOT, F_TAIL_UP0, F_CHUNK_UP, F_CHUNK_MID, F_CHUNK_DOWN, F_FWD_SEQ, F_REFINE_SEQ, F_REDO,
    F_MARK, F_RAGGED, F_RESOLVE, F_SQP, F_COUNT
};

// Optional per-launch timer (HIP events around each launch on its stream),
// installed by the ABI layer for the duration of a call.  `flops` is the
// algorithmic count of the launch (per-unit figures of Work below), `flops_min`
// the same with the combines counted at the minimal cost of the form the
// kernels execute (the Cholesky form, or the leaf form of the chunked sweeps).
struct Timer {
    virtual ~Timer() {}
    virtual void before(hipStream_t s, int fam, double flops, double bytes, double flops_min) = 0;
    virtual void after(hipStream_t s) = 0;
};
Timer*& current_timer();

template <typename K, typename... Args>
int launch_w(int nt, int fam, double flops, double bytes, double flops_min, K kernel, int64_t grid, hipStream_t s,
             Args... args) {
    if (grid <= 0) return LQR_OK;
    Timer* t = current_timer();
    if (t) t->before(s, fam, flops, bytes, flops_min);
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(nt), 0, s, args...);
    if (t) t->after(s);
    HIPCHK(hipGetLastError());
    return LQR_OK;
}

template <typename K, typename... Args>
int launch_nt(int nt, int fam, double flops, double bytes, K kernel, int64_t grid, hipStream_t s, Args... args) {
    return launch_w(nt, fam, flops, bytes, flops, kernel, grid, s, args...);
}

// grid of a task launch: one workgroup per task, except for the large-block
// engine whose workgroups loop over the tasks with one scratch slot each
template <class E>
inline int64_t task_grid(const Plan& p, int64_t tasks) {
    if (!E::BIG) return tasks;
    return tasks < p.big_grid ? tasks : p.big_grid;
}

// Algorithmic work per unit: flops counted as 2 per multiply-add; bytes =
// the records a unit must read and write once.  The combine counts are the
// per-unit figures of the method's cost model (general combine ~17 n^3, a
// combine with a complete suffix ~6.7 n^3, a forward map composition 2 n^3);
// comb_min / cheap_min are the minimal counts of the Cholesky form the
// kernels execute (67/6 n^3 and 31/6 n^3: two factorizations, the
// triangular solves and products at their triangular/symmetric cost),
// leaf_min that of the leaf form of a cheap combine (leaf_combine).
struct Work {
    double n, m, es, rec, srec, frec, vb, cb;
    explicit Work(const Plan& p, size_t esize)
        : n(p.n), m(p.m), es((double)esize), rec(p.rec), srec(p.srec), frec(p.frec),
          vb(p.leafv ? (double)p.n * p.m : 0.0), cb(p.noC ? (double)p.n * p.n : 0.0) {}
    double elem_f() const { return m * m * m / 3 + 2 * n * m * m + 4 * n * n * m - (cb > 0 ? n * n * m : 0.0); }
    // inputs read, the record written (with V, without C where the plan says so)
    double elem_b() const { return es * (2 * n * n + 2 * n * m + m * m + 2 * n + m + rec + vb - cb); }
    double comb_f() const { return 17.0 * n * n * n; }
    double comb_min() const { return 67.0 / 6.0 * n * n * n; }
    double comb_b() const { return es * 3 * rec; }
    double cheap_f() const { return 6.7 * n * n * n; }
    double cheap_min() const { return 31.0 / 6.0 * n * n * n; }
    double cheap_b() const { return es * (rec + 2 * srec); }
    // a cheap combine inside a sequential sweep: the suffix matrix it
    // extends was made by the step before and stays on chip, so only the
    // leaf, the suffix vector and the new suffix move (the first step of a
    // sweep also reads its n x n matrix: sweep_b)
    double seq_b() const { return es * (rec + srec + n); }
    double sweep_b() const { return es * n * n; }
    // the same step in the leaf form: the leaf without C, its n x m factor
    // V, the suffix vector, the new suffix; minimal flops of that form
    // (V'P2, V'P2V, the m x m factorization and solve, P2 - U'U, M A1,
    // A1'(M A1) at their symmetric/triangular cost)
    double leaf_b() const { return es * (2 * n * n + 2 * n + n * m + srec + n); }
    // a stage's inputs (A, B, Q, R, M, c, q, r): what a sweep that builds its
    // leaves reads per step besides the suffix it writes
    double elem_in_b() const { return es * (2 * n * n + 2 * n * m + m * m + 2 * n + m); }
    double leaf_min() const { return 3 * n * n * n + 3 * n * n * m + 2 * n * m * m + m * m * m / 3; }
    double pol_f() const { return 6 * n * n * m + 4 * n * m * m + m * m * m / 3; }
    double pol_b() const { return es * (n * n + 2 * n * m + m * m + 2 * n + m + srec + n * m + m + m * m + frec); }
    double fup_f() const { return 2 * n * n * n; }
    double fup_b() const { return es * 3 * frec; }
    double vec_f() const { return 2 * n * n; }
    double vec_b() const { return es * (frec + 2 * n); }
    double rec_f() const { return 2 * n * n + 2 * n * m; }
    double rec_b() const { return es * (srec + n * m + 2 * n + m); }
    // one stage of the sequential forward sweep: Abar x, K x, P x
    double fseq_f() const { return 4 * n * n + 2 * n * m; }
    double fseq_b() const { return es * (frec + n * m + m + srec + 2 * n + m); }
    // one stage of the sequential refinement sweep (backward + forward)
    double rseq_f() const { return 10 * n * n + 10 * n * m + 2 * m * m; }
    double rseq_b() const { return es * (2 * srec + 2 * frec + 2 * n * m + 2 * n * m + m * m + 8 * n + 4 * m); }
    double resid_f() const { return 2 * (3 * n * n + 4 * n * m + m * m); }
    double resid_b() const { return es * (2 * n * n + 2 * n * m + m * m + 6 * n + 2 * m); }
    double plain_f(int N) const { return N * (4 * n * n * n + 6 * n * n * m + 4 * n * m * m + m * m * m / 3); }
    double plain_b(int N) const { return es * N * (2 * n * n + 2 * n * m + m * m + 4 * n + m + n * n + n * m); }
};

#define LCHK(x)                    \
    do {                           \
        int rc_ = (x);             \
        if (rc_ != LQR_OK) return rc_; \
    } while (0)

// Buffers of a call beside the per-instance records.
struct Ctx {
    int32_t* active;   // [batch] refinement gating flags
    double* dws;       // FP64 partial sums of the residual, [batch * dstride + batch]
    double* ws64;      // FP64 redo slots (nullptr: no FP64 redo)
    Plan rp;           // plan of the redo slots (rp.batch = instances of the call)
    int redo_grid;     // workgroups (= slots) of the redo launch
};

// FP64 redo of the instances the FP32 solve marked (status bit 8), then the
// residual of their new solution (if the caller asked for residuals).
template <typename S, int TS>
int run_redo(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, const Ctx& cx,
             double* resid_out) {
    using E64 = EngOf<double, TS>;
    if (!cx.ws64) return LQR_OK;
    if constexpr (TS == kBigTS) {
        LCHK(launch_nt(E64::NT, F_REDO, 0, 0, k_redo_big<S, E64>, cx.redo_grid, s, cx.rp, in, out, cx.ws64));
    } else {
        LCHK(with_mb<TS>(p.m, [&](auto mb) {
            return launch_nt(64, F_REDO, 0, 0, k_redo<S, E64, decltype(mb)::value>, cx.redo_grid, s, cx.rp, in, out,
                             cx.ws64);
        }));
    }
    if (resid_out) {
        const int64_t Bi = p.batch;
        LCHK(launch_nt(256, F_MARK, 0, 0, k_mark_status<8>, (Bi + 255) / 256, s, (const int32_t*)out.status, cx.active, Bi));
        Plan pm = p;
        pm.active = cx.active;
        // one task unit per instance (the same sums in the same order as the
        // per-stage launch and its reduction): an instance that was not
        // redone leaves at its gate, so the launch costs a few microseconds
        LCHK(launch_nt(E64::NT, F_RESID, 0, 0, k_resid_inst<S, E64, false>, Bi, s, pm, in, (const S*)out.x,
                       (const S*)out.u, (const S*)out.lam, ws, cx.dws, resid_out, (int32_t*)nullptr, p.refine_tol,
                       (const int32_t*)out.status));
    }
    return LQR_OK;
}

// ----------------------------------------------------------------- solve
// The whole scan solve in one launch per instance batch (wavefront engine;
// plan.fused == 2), plus the FP64 redo launch over marked instances.  The
// flop and byte figures are those of the launch sequence it replaces.
template <typename S, int TS>
int run_fused(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, const Ctx& cx, int refine,
              double* resid_out, const Warm<S>& warm) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    static_assert(!E::BIG, "wavefront engine only");
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int N = p.N;
    double u_up = 0, u_down = 0, u_fup = 0;
    for (int l = 0; l + 1 < p.rt.nlev; ++l) u_up += p.rt.cnt[l] / 2, u_down += p.rt.cnt[l] / 2;
    for (int l = 0; l + 1 < p.ft.nlev; ++l) u_fup += p.ft.cnt[l] / 2;
    const double base = N * w.elem_f() + N * w.pol_f() + u_fup * w.fup_f();
    const double flops = B * (base + u_up * w.comb_f() + u_down * w.cheap_f());
    const double fmin = B * (base + u_up * w.comb_min() + u_down * w.cheap_min());
    const double bytes = B * (N * w.elem_b() + u_up * w.comb_b() + u_down * w.cheap_b() + N * w.pol_b() +
                              u_fup * w.fup_b());
    LCHK(with_mb<TS>(p.m, [&](auto mb) {
        constexpr int MB = decltype(mb)::value;
        return launch_w(64 * fused_waves<E>(), F_FUSED, flops, bytes, fmin, k_solve_fused<S, E, E64, MB>, p.batch, s,
                        p, in, out, ws, cx.dws, resid_out, warm, refine);
    }));
    return run_redo<S, TS>(p, s, in, out, ws, cx, resid_out);
}

template <typename S, int TS>
int run_scan(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, const Ctx& cx, int refine,
             double* resid_out, const Warm<S>& warm) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    constexpr int NT = E::NT;
    if constexpr (!E::BIG) {
        if (p.fused == 2) return run_fused<S, TS>(p, s, in, out, ws, cx, refine, resid_out, warm);
    }
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int64_t Bi = p.batch;
    const int N = p.N;
    int32_t* st = out.status;
    LCHK(launch_nt(256, F_CLEAR, 0, 4.0 * Bi, k_clear<int32_t>, (Bi + 255) / 256, s, st, Bi));
    // a1: elements
    // (the chunk-1 sweep that builds its leaves itself needs no element launch)
    if (!p.fuse_elem) {
        LCHK(with_mb<TS>(p.m, [&](auto mb) {
            constexpr int MB = decltype(mb)::value;
            return launch_nt(NT, F_ELEM, B * N * w.elem_f(), B * N * w.elem_b(), k_element<S, E, MB>,
                             task_grid<E>(p, Bi * (N + 1)), s, p, in, ws, st);
        }));
    }
    // a3: reverse scan
    if (p.sched == 0) {
        // balanced tree: up-sweep, root, down-sweep
        for (int l = 0; l + 1 < p.rt.nlev; ++l) {
            const double u = B * (p.rt.cnt[l] / 2);
            LCHK(launch_w(NT, F_UP, u * w.comb_f(), u * w.comb_b(), u * w.comb_min(), k_up<S, E>,
                          task_grid<E>(p, Bi * p.rt.cnt[l + 1]), s, p, ws, l, st));
        }
        LCHK(launch_nt(WG, F_ROOT, 0, 2 * B * w.es * p.srec, k_root<S>, Bi, s, p, ws));
        for (int l = p.rt.nlev - 2; l >= 0; --l) {
            const int h = down_half(p, l);
            const double u = B * h;
            LCHK(launch_w(NT, F_DOWN, u * w.cheap_f(), u * w.cheap_b(), u * w.cheap_min(), k_down<S, E>,
                          task_grid<E>(p, Bi * h), s, p, ws, l, st));
        }
    } else if constexpr (!E::BIG) {
        const double ut = B * (N - p.tail);   // cheap combines of the sequential sweep
        if (p.sched == 1) {
            // split: the sweep and the first up-sweep level of the head tree
            // side by side, the rest of the head tree, its root with the
            // sweep's suffix, the head's down-sweep
            const int c0 = up_count(p, 0);
            const double u0 = B * c0;
            LCHK(launch_w(NT, F_TAIL_UP0, ut * w.cheap_f() + u0 * w.comb_f(), ut * w.cheap_b() + u0 * w.comb_b(),
                          ut * w.cheap_min() + u0 * w.comb_min(), k_tail_up0<S, E>, Bi + Bi * c0, s, p, ws, st));
            for (int l = 1; l + 1 < p.rt.nlev; ++l) {
                const int c = up_count(p, l);
                if (c == 0) continue;
                const double u = B * c;
                LCHK(launch_w(NT, F_UP, u * w.comb_f(), u * w.comb_b(), u * w.comb_min(), k_up<S, E>, Bi * c, s, p,
                              ws, l, st));
            }
            LCHK(launch_w(NT, F_TROOT, B * w.cheap_f(), B * w.cheap_b(), B * w.cheap_min(), k_tail_root<S, E>, Bi, s,
                          p, ws, st));
            for (int l = p.rt.nlev - 2; l >= 0; --l) {
                const int h = down_half(p, l);
                if (h == 0) continue;
                const double u = B * h;
                LCHK(launch_w(NT, F_DOWN, u * w.cheap_f(), u * w.cheap_b(), u * w.cheap_min(), k_down<S, E>, Bi * h,
                              s, p, ws, l, st));
            }
        } else if (p.fuse_elem) {
            // chunk length 1, leaves built in the sweep: one launch for the
            // whole reverse scan (elements included)
            const double u = B * N;
            LCHK(with_lw<TS>(p, [&](auto lw) {
                constexpr int LW = decltype(lw)::value;
                if constexpr (LW > 0 && 2 * LW <= TS) {
                    return launch_w(NT, F_CHUNK_MID, u * (w.cheap_f() + w.elem_f()),
                                    u * (w.elem_in_b() + w.es * p.srec) + B * w.es * 2 * p.srec,
                                    u * (w.leaf_min() + w.elem_f()), k_chunk_mid_elem<S, E, LW>, Bi, s, p, in, ws,
                                    st);
                } else {
                    return (int)fail(LQR_EUNSUPPORTED, "leaf-building sweep planned for an unsupported shape");
                }
            }));
        } else {
            // chunked: chunk aggregates beside the sweep, suffixes at the
            // chunk starts, then the other leaves of every chunk
            const double ug = B * (p.tail - p.nchunk);   // general combines of the aggregates
            // chunks of one leaf have no aggregate to form: at chunk length 1
            // the launch holds the sweep tasks only
            const int64_t agg_tasks = p.chunk == 1 ? 0 : Bi * p.nchunk;
            LCHK(launch_w(NT, F_CHUNK_UP, ut * w.cheap_f() + ug * w.comb_f(), ut * w.cheap_b() + ug * w.comb_b(),
                          ut * w.cheap_min() + ug * w.comb_min(), k_chunk_up<S, E>, Bi + agg_tasks, s, p, ws, st));
            if (p.nchunk > 0) {
                const double um = B * p.nchunk, ud = B * (p.tail - p.nchunk);
                int down_sweeps = 0;   // chunks with at least one leaf after their start
                for (int c = 0; c < p.nchunk; ++c) down_sweeps += chunk_end(p, c) - c * p.chunk >= 2;
                LCHK(with_lw<TS>(p, [&](auto lw) {
                    constexpr int LW = decltype(lw)::value;
                    // phase 2 in the leaf form only when every chunk is one leaf
                    if (LW > 0 && p.chunk == 1) {
                        LCHK(launch_w(NT, F_CHUNK_MID, um * w.cheap_f(), um * w.leaf_b() + B * w.sweep_b(),
                                      um * w.leaf_min(), k_chunk_mid<S, E, LW>, Bi, s, p, ws, st));
                    } else {
                        LCHK(launch_w(NT, F_CHUNK_MID, um * w.cheap_f(), um * w.seq_b() + B * w.sweep_b(),
                                      um * w.cheap_min(), k_chunk_mid<S, E, 0>, Bi, s, p, ws, st));
                    }
                    // no chunk with a leaf after its start: nothing for phase 3
                    if (down_sweeps == 0) return (int)LQR_OK;
                    return launch_w(NT, F_CHUNK_DOWN, ud * w.cheap_f(),
                                    ud * (LW > 0 ? w.leaf_b() : w.seq_b()) + B * down_sweeps * w.sweep_b(),
                                    ud * (LW > 0 ? w.leaf_min() : w.cheap_min()), k_chunk_down<S, E, LW>,
                                    Bi * p.nchunk, s, p, ws, st);
                }));
            }
        }
    }
    // a4: policy and closed-loop maps
    LCHK(with_mb<TS>(p.m, [&](auto mb) {
        constexpr int MB = decltype(mb)::value;
        return launch_nt(NT, F_POLICY, B * N * w.pol_f(), B * N * w.pol_b(), k_policy<S, E, MB>,
                         task_grid<E>(p, Bi * N), s, p, in, ws, st);
    }));
    // a5: forward scan of the closed-loop maps (matrix part of the tree)
    if (!p.fwdseq) {
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FUP, u * w.fup_f(), u * w.fup_b(), k_fup<S, E, false>, Bi * p.ft.cnt[l + 1], s, p,
                           ws, l));
        }
    }
    const double fwd_nodes = B * (double)(p.ft.total - p.ft.cnt[p.ft.nlev - 1]);
    if (warm.x) {
        // warm start: the outputs start at the given solution and the
        // refinement sweeps below correct it with the factors just computed
        const int64_t cx_ = Bi * (N + 1) * p.n, cu = Bi * N * p.m;
        auto cp = [&](const S* src, S* dst, int64_t count) -> int {
            if (src == dst) return LQR_OK;
            const int64_t g = (count + 255) / 256;
            return launch_nt(256, F_WARM, 0, 2.0 * w.es * count, k_copy<S>, g < 4096 ? g : 4096, s, src, dst,
                             count);
        };
        LCHK(cp(warm.x, out.x, cx_));
        LCHK(cp(warm.u, out.u, cu));
        LCHK(cp(warm.lam, out.lam, cx_));
        if (refine < 1) refine = 1;
    } else if (p.fwdseq) {
        // a5 + a6 as one sequential sweep per instance
        LCHK(launch_nt(NT, F_FWD_SEQ, B * N * w.fseq_f(), B * N * w.fseq_b(), k_fwd_seq<S, E>, Bi, s, p, ws, in.x0,
                       out));
    } else if (p.fused) {
        // a5 down-sweep + a6 per instance
        LCHK(launch_nt(NT, F_FWD_INST, fwd_nodes * w.vec_f() + B * (N + 1) * w.rec_f(),
                       fwd_nodes * w.vec_b() + B * (N + 1) * w.rec_b(), k_fwd_inst<S, E>, Bi, s, p, ws, in.x0,
                       (int64_t)p.n, out));
    } else {
        LCHK(launch_nt(WG, F_FROOT, 0, 2 * B * w.es * p.n, k_froot<S>, Bi, s, p, ws, in.x0, (int64_t)p.n));
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FDOWN, u * w.vec_f(), u * w.vec_b(), k_fdown<S, E>, Bi * p.ft.cnt[l], s, p, ws, l));
        }
        // a6: controls and costates
        LCHK(launch_nt(NT, F_RECOVER, B * (N + 1) * w.rec_f(), B * (N + 1) * w.rec_b(), k_recover<S, E, false>,
                       Bi * (N + 1), s, p, ws, out));
    }
    // a7: FP64 residual + refinement sweeps, each for the instances whose
    // residual is above the tolerance (never those marked for the FP64 redo)
    int32_t* active = cx.active;
    double* rel = resid_out ? resid_out : cx.dws + Bi * p.dstride;
    Plan pg = p;
    const double ref_f = B * N * 7 * w.vec_f() + 2 * fwd_nodes * w.vec_f() * 2 + B * (N + 1) * w.rec_f();
    const double ref_b = B * N * 7 * w.vec_b() + 2 * fwd_nodes * w.vec_b() * 2 + B * (N + 1) * w.rec_b();
    const double rf = B * (N + 1) * w.resid_f(), rb = B * (N + 1) * w.resid_b();
    for (int sw = 0; sw < refine; ++sw) {
        // the first decision covers every instance, later ones revisit the
        // instances the previous sweep corrected
        const Plan& pr = sw >= 1 ? pg : p;
        if (p.fused && !p.fwdseq) {
            LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid_inst<S, E64, true>, Bi, s, pr, in, (const S*)out.x,
                           (const S*)out.u, (const S*)out.lam, ws, cx.dws, rel, active, p.refine_tol,
                           (const int32_t*)st));
            pg.active = active;
            LCHK(launch_nt(NT, F_REFINE_INST, ref_f, ref_b, k_refine_inst<S, E>, Bi, s, pg, in, ws, out));
            continue;
        }
        LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid<S, E64, true>, Bi * (N + 1), s, pr, in, (const S*)out.x,
                       (const S*)out.u, (const S*)out.lam, ws, cx.dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pr,
                       (const double*)cx.dws, rel, active, p.refine_tol, (const int32_t*)st));
        pg.active = active;
        if (p.fwdseq) {
            LCHK(launch_nt(NT, F_REFINE_SEQ, B * N * w.rseq_f(), B * N * w.rseq_b(), k_refine_seq<S, E>, Bi, s, pg,
                           in, ws, out));
            continue;
        }
        LCHK(launch_nt(NT, F_REF_D, B * N * 3 * w.vec_f(), B * N * 3 * w.vec_b(), k_ref_d<S, E>, Bi * N, s, pg, ws));
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_BUP, u * w.vec_f(), u * w.vec_b(), k_bvec_up<S, E>, Bi * p.ft.cnt[l + 1], s, pg, ws,
                           l));
        }
        LCHK(launch_nt(WG, F_BROOT, 0, 4 * B * w.es * p.n, k_broot<S>, Bi, s, pg, ws));
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_BDOWN, u * w.vec_f(), u * w.vec_b(), k_bvec_down<S, E>, Bi * p.ft.cnt[l], s, pg, ws,
                           l));
        }
        LCHK(launch_nt(NT, F_REF_KFF, B * N * 4 * w.vec_f(), B * N * 4 * w.vec_b(), k_ref_kff<S, E>, Bi * N, s, pg,
                       in, ws));
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FUPV, u * w.vec_f(), u * w.vec_b(), k_fup<S, E, true>, Bi * p.ft.cnt[l + 1], s, pg,
                           ws, l));
        }
        LCHK(launch_nt(WG, F_FROOT, 0, 2 * B * w.es * p.n, k_froot<S>, Bi, s, pg, ws, (const S*)(ws + p.o_x0p),
                       p.stride));
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FDOWN, u * w.vec_f(), u * w.vec_b(), k_fdown<S, E>, Bi * p.ft.cnt[l], s, pg, ws, l));
        }
        LCHK(launch_nt(NT, F_RECOVER_ADD, B * (N + 1) * w.rec_f(), B * (N + 1) * w.rec_b(), k_recover<S, E, true>,
                       Bi * (N + 1), s, pg, ws, out));
    }
    if (resid_out) {
        // after an adaptive sweep only the instances it touched changed
        if (p.fused && !p.fwdseq) {
            LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid_inst<S, E64, false>, Bi, s, pg, in, (const S*)out.x,
                           (const S*)out.u, (const S*)out.lam, ws, cx.dws, resid_out, (int32_t*)nullptr,
                           p.refine_tol, (const int32_t*)st));
        } else {
            LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid<S, E64, false>, Bi * (N + 1), s, pg, in, (const S*)out.x,
                           (const S*)out.u, (const S*)out.lam, ws, cx.dws));
            LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pg,
                           (const double*)cx.dws, resid_out, (int32_t*)nullptr, p.refine_tol, (const int32_t*)st));
        }
    }
    return run_redo<S, TS>(p, s, in, out, ws, cx, resid_out);
}

// Re-solve with the factors the last scan solve of these matrices left in
// the workspace (new x0, c, q, r): one backward + forward vector sweep per
// instance, the FP64 residual and refinement sweeps as in run_scan, then
// the FP64 redo of the instances the last solve marked (bit 8 of the
// incoming status words).
template <typename S, int TS>
int run_resolve(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, const Ctx& cx, int refine,
                double* resid_out) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    constexpr int NT = E::NT;
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int64_t Bi = p.batch;
    const int N = p.N;
    int32_t* st = out.status;
    LCHK(launch_nt(NT, F_RESOLVE, B * N * w.rseq_f(), B * N * w.rseq_b(), k_resolve_seq<S, E>, Bi, s, p, in, ws,
                   out));
    int32_t* active = cx.active;
    double* rel = resid_out ? resid_out : cx.dws + Bi * p.dstride;
    Plan pg = p;
    const double rf = B * (N + 1) * w.resid_f(), rb = B * (N + 1) * w.resid_b();
    for (int sw = 0; sw < refine; ++sw) {
        const Plan& pr = sw >= 1 ? pg : p;
        LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid<S, E64, true>, Bi * (N + 1), s, pr, in, (const S*)out.x,
                       (const S*)out.u, (const S*)out.lam, ws, cx.dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pr,
                       (const double*)cx.dws, rel, active, p.refine_tol, (const int32_t*)st));
        pg.active = active;
        LCHK(launch_nt(NT, F_REFINE_SEQ, B * N * w.rseq_f(), B * N * w.rseq_b(), k_refine_seq<S, E>, Bi, s, pg, in,
                       ws, out));
    }
    if (resid_out) {
        LCHK(launch_nt(NT, F_RESID, rf, rb, k_resid<S, E64, false>, Bi * (N + 1), s, pg, in, (const S*)out.x,
                       (const S*)out.u, (const S*)out.lam, ws, cx.dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pg,
                       (const double*)cx.dws, resid_out, (int32_t*)nullptr, p.refine_tol, (const int32_t*)st));
    }
    return run_redo<S, TS>(p, s, in, out, ws, cx, resid_out);
}

template <typename S, int TS>
int run_plain(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, const Ctx& cx,
              double* resid_out) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    constexpr int NT = E64::NT;
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int64_t Bi = p.batch;
    LCHK(launch_nt(256, F_CLEAR, 0, 4.0 * B, k_clear<int32_t>, (Bi + 255) / 256, s, out.status, Bi));
    if constexpr (E::BIG)
        LCHK(launch_nt(NT, F_PLAIN, B * w.plain_f(p.N), B * w.plain_b(p.N), k_plain_big<S, E>, task_grid<E>(p, Bi), s,
                       p, in, out, ws));
    else
        LCHK(with_mb<TS>(p.m, [&](auto mb) {
            return launch_nt(NT, F_PLAIN, B * w.plain_f(p.N), B * w.plain_b(p.N), k_plain<S, E, decltype(mb)::value>,
                             Bi, s, p, in, out, ws);
        }));
    if (resid_out) {
        LCHK(launch_nt(NT, F_RESID, B * (p.N + 1) * w.resid_f(), B * (p.N + 1) * w.resid_b(), k_resid<S, E64, false>,
                       Bi * (p.N + 1), s, p, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, cx.dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (p.N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, p,
                       (const double*)cx.dws, resid_out, (int32_t*)nullptr, p.refine_tol, (const int32_t*)nullptr));
    }
    return LQR_OK;
}

template <typename S, int TS>
int run_resid(const Plan& p, hipStream_t s, const In<S>& in, const S* x, const S* u, const S* lam, S* ws,
              double* dws, double* rel) {
    using E64 = EngOf<double, TS>;
    constexpr int NT = E64::NT;
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    LCHK(launch_nt(NT, F_RESID, B * (p.N + 1) * w.resid_f(), B * (p.N + 1) * w.resid_b(), k_resid<S, E64, false>,
                   p.batch * (p.N + 1), s, p, in, x, u, lam, ws, dws));
    LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (p.N + 1), k_resid_reduce<double>, (p.batch + 63) / 64, s, p,
                   (const double*)dws, rel, (int32_t*)nullptr, p.refine_tol, (const int32_t*)nullptr));
    return LQR_OK;
}

// Ragged batch from a device descriptor table, the problems of one padded
// order class: the persistent one-launch solve over `slots` workgroups,
// then the FP64 redo of the problems it marked (ragged_redo_slots workgroups).
template <typename S, int TS>
int run_ragged(hipStream_t s, const RaggedArgs<S>& a, int slots, int redo_slots, int32_t* counters) {
    if constexpr (TS == kBigTS) {
        return fail(LQR_EUNSUPPORTED, "the ragged persistent solve runs on the wavefront engine");
    } else {
        using E = EngOf<S, TS>;
        using E64 = EngOf<double, TS>;
        RaggedArgs<S> af = a;
        af.counter = counters;
        LCHK(launch_nt(64 * fused_waves<E>(), F_RAGGED, 0, 0, k_ragged_fused<S, E, E64>, slots, s, af));
        if (a.fallback && redo_slots > 0) {
            RaggedArgs<S> ar = a;
            ar.counter = counters + 1;
            LCHK(launch_nt(64, F_REDO, 0, 0, k_ragged_redo<S, E64>, redo_slots, s, ar));
        }
        return LQR_OK;
    }
}

// explicit instantiation per (padded-order class, storage type): each pair
// is its own translation unit (inst.hip), so the classes compile in parallel
#define LQR_RUNS(PREFIX, TSV, SV)                                                                              \
    PREFIX template int run_scan<SV, TSV>(const Plan&, hipStream_t, const In<SV>&, const Out<SV>&, SV*,         \
                                          const Ctx&, int, double*, const Warm<SV>&);                          \
    PREFIX template int run_plain<SV, TSV>(const Plan&, hipStream_t, const In<SV>&, const Out<SV>&, SV*,        \
                                           const Ctx&, double*);                                               \
    PREFIX template int run_resid<SV, TSV>(const Plan&, hipStream_t, const In<SV>&, const SV*, const SV*,       \
                                           const SV*, SV*, double*, double*);                                  \
    PREFIX template int run_ragged<SV, TSV>(hipStream_t, const RaggedArgs<SV>&, int, int, int32_t*);         \
    PREFIX template int run_resolve<SV, TSV>(const Plan&, hipStream_t, const In<SV>&, const Out<SV>&, SV*,      \
                                             const Ctx&, int, double*);

#define LQR_DECLARE_RUNS(TSV) LQR_RUNS(extern, TSV, float) LQR_RUNS(extern, TSV, double)
#define LQR_DEFINE_RUNS(TSV, SV) LQR_RUNS(, TSV, SV)

}  // namespace lqr
