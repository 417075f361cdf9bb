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
    F_CLEAR, F_ELEM, F_ELEM_FB, F_UP, F_ROOT, F_DOWN, F_POLICY, F_POLICY_FB, F_FUP, F_FROOT, F_FDOWN,
    F_RECOVER, F_RESID, F_REF_D, F_BUP, F_BROOT, F_BDOWN, F_REF_KFF, F_FUPV, F_RECOVER_ADD, F_REDUCE,
    F_PLAIN, F_UP_FB, F_DOWN_FB, F_FWD_INST, F_REFINE_INST, F_WARM, F_PACK, F_FUSED, F_FUSED_FB, F_TAIL, F_TAIL_FB,
    F_TROOT, F_TROOT_FB, F_TAIL_UP0, F_COUNT
};

// Optional per-launch timer (HIP events around each launch on its stream),
// installed by the ABI layer for the duration of a call.
struct Timer {
    virtual ~Timer() {}
    virtual void before(hipStream_t s, int fam, double flops, double bytes) = 0;
    virtual void after(hipStream_t s) = 0;
};
Timer*& current_timer();

template <typename K, typename... Args>
int launch_nt(int nt, int fam, double flops, double bytes, K kernel, int64_t grid, hipStream_t s, Args... args) {
    if (grid <= 0) return LQR_OK;
    Timer* t = current_timer();
    if (t) t->before(s, fam, flops, bytes);
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3(nt), 0, s, args...);
    if (t) t->after(s);
    HIPCHK(hipGetLastError());
    return LQR_OK;
}

// Layout of the int32 workspace: queue counters, then one id list per
// (family, level) with room for every task of that launch.
constexpr int kQElem = 0, kQPolicy = 1, kQUp = 2, kQDown = 2 + LQR_MAXLEV, kQTail = 2 + 2 * LQR_MAXLEV,
              kQTailRoot = kQTail + 1, kQCount = 64;
static_assert(kQTailRoot < kQCount, "queue counters");
struct Queues {
    int64_t list[kQCount];   // offsets (int32 elements) of each list
    int64_t total;
};
inline Queues queue_layout(const Plan& p) {
    Queues q;
    for (int i = 0; i < kQCount; ++i) q.list[i] = 0;
    int64_t off = kQCount;
    auto add = [&](int idx, int64_t n) { q.list[idx] = off; off += (n + 63) / 64 * 64; };
    add(kQElem, p.batch * (p.N + 1));
    add(kQPolicy, p.batch * p.N);
    for (int l = 0; l + 1 < p.rt.nlev; ++l) add(kQUp + l, p.batch * p.rt.cnt[l + 1]);
    for (int l = 0; l + 1 < p.rt.nlev; ++l) add(kQDown + l, p.batch * (p.rt.cnt[l] / 2));
    add(kQTail, p.batch);
    add(kQTailRoot, p.batch);
    q.total = off;
    return q;
}
inline FbQueue fbq(int32_t* iws, const Queues& q, int idx) { return FbQueue{iws + idx, iws + q.list[idx]}; }
inline int64_t drain_grid(int64_t tasks) { return tasks < 1024 ? tasks : 1024; }

// grid of a task launch: one workgroup per task, except for the large-block
// engine whose workgroups loop over the tasks with one scratch slot each
template <class E>
inline int64_t task_grid(const Plan& p, int64_t tasks) {
    if (!E::BIG) return tasks;
    return tasks < p.big_grid ? tasks : p.big_grid;
}
template <class E>
inline int64_t fb_grid(const Plan& p, int64_t tasks) {
    const int64_t g = drain_grid(tasks);
    return E::BIG && g > p.big_grid ? p.big_grid : g;
}

// Algorithmic work per unit (flops counted as 2 per multiply-add, the
// symmetric and triangular products at their minimal cost; bytes = the
// records a unit must read and write once).
struct Work {
    double n, m, es, rec, srec, frec;
    explicit Work(const Plan& p, size_t esize)
        : n(p.n), m(p.m), es((double)esize), rec(p.rec), srec(p.srec), frec(p.frec) {}
    double elem_f() const { return m * m * m / 3 + 2 * n * m * m + 4 * n * n * m; }
    double elem_b() const { return es * (2 * n * n + 2 * n * m + m * m + 2 * n + m + rec); }
    double comb_f() const { return 67.0 / 6.0 * n * n * n; }          // general combine
    double comb_b() const { return es * 3 * rec; }
    double cheap_f() const { return 31.0 / 6.0 * n * n * n; }         // combine with a complete suffix
    double cheap_b() const { return es * (rec + 2 * srec); }
    double pol_f() const { return 6 * n * n * m + 4 * n * m * m + m * m * m / 3; }
    double pol_b() const { return es * (n * n + 2 * n * m + m * m + 2 * n + m + srec + n * m + m + m * m + frec); }
    double fup_f() const { return 2 * n * n * n; }
    double fup_b() const { return es * 3 * frec; }
    double vec_f() const { return 2 * n * n; }
    double vec_b() const { return es * (frec + 2 * n); }
    double rec_f() const { return 2 * n * n + 2 * n * m; }
    double rec_b() const { return es * (srec + n * m + 2 * n + m); }
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

// ----------------------------------------------------------------- solve
// The whole scan solve in one launch per instance batch (wavefront engine;
// plan.fused == 2), plus the FP64 redo launch over flagged instances.  The
// flop and byte figures are those of the launch sequence it replaces.
template <typename S, int TS>
int run_fused(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, double* dws, int refine,
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
    const double flops = B * (N * w.elem_f() + u_up * w.comb_f() + u_down * w.cheap_f() + N * w.pol_f() +
                              u_fup * w.fup_f());
    const double bytes = B * (N * w.elem_b() + u_up * w.comb_b() + u_down * w.cheap_b() + N * w.pol_b() +
                              u_fup * w.fup_b());
    return with_mb<TS>(p.m, [&](auto mb) {
        constexpr int MB = decltype(mb)::value;
        LCHK(launch_nt(64 * fused_waves<E>(), F_FUSED, flops, bytes, k_solve_fused<S, E, E64, MB, false>, p.batch,
                       s, p, in, out, ws, dws, resid_out, warm, refine));
        if constexpr (sizeof(S) == 4) {
            if (p.fallback) {
                Plan pf = p;
                pf.fallback = 0;
                LCHK(launch_nt(64 * fused_waves<E64>(), F_FUSED_FB, 0, 0, k_solve_fused<S, E64, E64, MB, true>,
                               p.batch, s, pf, in, out, ws, dws, resid_out, warm, refine));
            }
        }
        return LQR_OK;
    });
}

template <typename S, int TS>
int run_scan(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, int32_t* iws,
             double* dws, int refine, double* resid_out, const Warm<S>& warm) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    constexpr int NT = E::NT;
    if constexpr (!E::BIG) {
        if (p.fused == 2) return run_fused<S, TS>(p, s, in, out, ws, dws, refine, resid_out, warm);
    }
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int64_t Bi = p.batch;
    const int N = p.N;
    const Queues Qs = queue_layout(p);
    const bool fb = sizeof(S) == 4 && p.fallback;
    LCHK(launch_nt(WG, F_CLEAR, 0, 4.0 * Bi, k_clear<int32_t>, (Bi + 255) / 256 * 4, s, out.status, Bi, iws,
                (int64_t)kQCount));
    // a1: elements (+ FP64 redo of queued stages)
    {
        const FbQueue q = fbq(iws, Qs, kQElem);
        LCHK(with_mb<TS>(p.m, [&](auto mb) {
            constexpr int MB = decltype(mb)::value;
            LCHK(launch_nt(NT, F_ELEM, B * N * w.elem_f(), B * N * w.elem_b(), k_element<S, E, false, MB>,
                           task_grid<E>(p, Bi * (N + 1)), s, p, in, ws, out.status, q));
            if (fb)
                LCHK(launch_nt(NT, F_ELEM_FB, 0, 0, k_element<S, E64, true, MB>, fb_grid<E64>(p, Bi * (N + 1)), s, p,
                               in, ws, out.status, q));
            return LQR_OK;
        }));
    }
    // a3: reverse scan, up-sweep then down-sweep (split schedule: the
    // sequential sweep of the tail leaves first, the tree over the head)
    int l_first = 0;   // first up-sweep level launched by the loop below
    if constexpr (!E::BIG) {
        if (p.tail) {
            const double u = B * (N - p.tail);
            const FbQueue q = fbq(iws, Qs, kQTail);
            const int c0 = up_count(p, 0);
            if (c0 > 0) {
                // the sweeps and the first up-sweep level side by side
                const double u0 = B * c0;
                const FbQueue q0 = fbq(iws, Qs, kQUp);
                LCHK(launch_nt(NT, F_TAIL_UP0, u * w.cheap_f() + u0 * w.comb_f(), u * w.cheap_b() + u0 * w.comb_b(),
                               k_tail_up0<S, E>, Bi + Bi * c0, s, p, ws, out.status, q, q0));
                if (fb) {
                    LCHK(launch_nt(NT, F_TAIL_FB, 0, 0, k_tail<S, E64, true>, fb_grid<E64>(p, Bi), s, p, ws,
                                   out.status, q));
                    LCHK(launch_nt(NT, F_UP_FB, 0, 0, k_up<S, E64, true>, fb_grid<E64>(p, Bi * c0), s, p, ws, 0,
                                   out.status, q0));
                }
                l_first = 1;
            } else {
                LCHK(launch_nt(NT, F_TAIL, u * w.cheap_f(), u * w.cheap_b(), k_tail<S, E, false>, Bi, s, p, ws,
                               out.status, q));
                if (fb)
                    LCHK(launch_nt(NT, F_TAIL_FB, 0, 0, k_tail<S, E64, true>, fb_grid<E64>(p, Bi), s, p, ws,
                                   out.status, q));
            }
        }
    }
    for (int l = l_first; l + 1 < p.rt.nlev; ++l) {
        const int c = up_count(p, l);
        if (c == 0) continue;
        const double u = B * (p.tail ? c : p.rt.cnt[l] / 2);
        const FbQueue q = fbq(iws, Qs, kQUp + l);
        LCHK(launch_nt(NT, F_UP, u * w.comb_f(), u * w.comb_b(), k_up<S, E, false>, task_grid<E>(p, Bi * c), s, p, ws, l,
                    out.status, q));
        if (fb)
            LCHK(launch_nt(NT, F_UP_FB, 0, 0, k_up<S, E64, true>, fb_grid<E64>(p, Bi * c), s, p, ws, l,
                        out.status, q));
    }
    if (!p.tail) {
        LCHK(launch_nt(WG, F_ROOT, 0, 2 * B * w.es * p.srec, k_root<S>, Bi, s, p, ws));
    } else if constexpr (!E::BIG) {
        const FbQueue q = fbq(iws, Qs, kQTailRoot);
        LCHK(launch_nt(NT, F_TROOT, B * w.cheap_f(), B * w.cheap_b(), k_tail_root<S, E, false>, Bi, s, p, ws,
                       out.status, q));
        if (fb)
            LCHK(launch_nt(NT, F_TROOT_FB, 0, 0, k_tail_root<S, E64, true>, fb_grid<E64>(p, Bi), s, p, ws, out.status,
                           q));
    }
    for (int l = p.rt.nlev - 2; l >= 0; --l) {
        const int h = down_half(p, l);
        if (h == 0) continue;
        const double u = B * h;
        const FbQueue q = fbq(iws, Qs, kQDown + l);
        LCHK(launch_nt(NT, F_DOWN, u * w.cheap_f(), u * w.cheap_b(), k_down<S, E, false>, task_grid<E>(p, Bi * h), s, p,
                    ws, l, out.status, q));
        if (fb)
            LCHK(launch_nt(NT, F_DOWN_FB, 0, 0, k_down<S, E64, true>, fb_grid<E64>(p, Bi * h), s, p, ws, l,
                        out.status, q));
    }
    // a4: policy and closed-loop maps
    {
        const FbQueue q = fbq(iws, Qs, kQPolicy);
        LCHK(with_mb<TS>(p.m, [&](auto mb) {
            constexpr int MB = decltype(mb)::value;
            LCHK(launch_nt(NT, F_POLICY, B * N * w.pol_f(), B * N * w.pol_b(), k_policy<S, E, false, MB>,
                           task_grid<E>(p, Bi * N), s, p, in, ws, out.status, q));
            if (fb)
                LCHK(launch_nt(NT, F_POLICY_FB, 0, 0, k_policy<S, E64, true, MB>, fb_grid<E64>(p, Bi * N), s, p, in,
                               ws, out.status, q));
            return LQR_OK;
        }));
    }
    // a5: forward scan of the closed-loop maps
    for (int l = 0; l + 1 < p.ft.nlev; ++l) {
        const double u = B * (p.ft.cnt[l] / 2);
        LCHK(launch_nt(NT, F_FUP, u * w.fup_f(), u * w.fup_b(), k_fup<S, E, false>, Bi * p.ft.cnt[l + 1], s, p, ws, l));
    }
    const double fwd_nodes = B * (double)(p.ft.total - p.ft.cnt[p.ft.nlev - 1]);
    if (warm.x) {
        // warm start: the outputs start at the given solution and the
        // refinement sweeps below correct it with the factors just computed
        const int64_t cx = Bi * (N + 1) * p.n, cu = Bi * N * p.m;
        auto cp = [&](const S* src, S* dst, int64_t count) -> int {
            if (src == dst) return LQR_OK;
            const int64_t g = (count + 255) / 256;
            return launch_nt(256, F_WARM, 0, 2.0 * w.es * count, k_copy<S>, g < 4096 ? g : 4096, s, src, dst,
                             count);
        };
        LCHK(cp(warm.x, out.x, cx));
        LCHK(cp(warm.u, out.u, cu));
        LCHK(cp(warm.lam, out.lam, cx));
        if (refine < 1) refine = 1;
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
    // a7: FP64 residual + refinement sweeps (the second only for instances
    // whose residual after the first is still above the tolerance)
    int32_t* active = iws + Qs.total;
    double* rel = resid_out ? resid_out : dws + Bi * p.dstride;
    Plan pg = p;
    const double ref_f = B * N * 7 * w.vec_f() + 2 * fwd_nodes * w.vec_f() * 2 + B * (N + 1) * w.rec_f();
    const double ref_b = B * N * 7 * w.vec_b() + 2 * fwd_nodes * w.vec_b() * 2 + B * (N + 1) * w.rec_b();
    for (int sw = 0; sw < refine; ++sw) {
        // every sweep runs only for the instances whose residual is above
        // the tolerance: the first decision covers every instance, later
        // ones revisit the instances the previous sweep corrected
        const Plan& pr = sw >= 1 ? pg : p;
        if (p.fused) {
            LCHK(launch_nt(NT, F_RESID, B * (N + 1) * w.resid_f(), B * (N + 1) * w.resid_b(), k_resid_inst<S, E64, true>,
                        Bi, s, pr, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws, rel, active,
                        p.refine_tol));
            pg.active = active;
            LCHK(launch_nt(NT, F_REFINE_INST, ref_f, ref_b, k_refine_inst<S, E>, Bi, s, pg, in, ws, out));
            continue;
        }
        LCHK(launch_nt(NT, F_RESID, B * (N + 1) * w.resid_f(), B * (N + 1) * w.resid_b(), k_resid<S, E64, true>,
                    Bi * (N + 1), s, pr, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pr,
                       (const double*)dws, rel, active, p.refine_tol));
        pg.active = active;
        LCHK(launch_nt(NT, F_REF_D, B * N * 3 * w.vec_f(), B * N * 3 * w.vec_b(), k_ref_d<S, E>, Bi * N, s, pg, ws));
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_BUP, u * w.vec_f(), u * w.vec_b(), k_bvec_up<S, E>, Bi * p.ft.cnt[l + 1], s, pg, ws, l));
        }
        LCHK(launch_nt(WG, F_BROOT, 0, 4 * B * w.es * p.n, k_broot<S>, Bi, s, pg, ws));
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_BDOWN, u * w.vec_f(), u * w.vec_b(), k_bvec_down<S, E>, Bi * p.ft.cnt[l], s, pg, ws, l));
        }
        LCHK(launch_nt(NT, F_REF_KFF, B * N * 4 * w.vec_f(), B * N * 4 * w.vec_b(), k_ref_kff<S, E>, Bi * N, s, pg, in, ws));
        for (int l = 0; l + 1 < p.ft.nlev; ++l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FUPV, u * w.vec_f(), u * w.vec_b(), k_fup<S, E, true>, Bi * p.ft.cnt[l + 1], s, pg, ws, l));
        }
        LCHK(launch_nt(WG, F_FROOT, 0, 2 * B * w.es * p.n, k_froot<S>, Bi, s, pg, ws, (const S*)(ws + p.o_x0p), p.stride));
        for (int l = p.ft.nlev - 2; l >= 0; --l) {
            const double u = B * (p.ft.cnt[l] / 2);
            LCHK(launch_nt(NT, F_FDOWN, u * w.vec_f(), u * w.vec_b(), k_fdown<S, E>, Bi * p.ft.cnt[l], s, pg, ws, l));
        }
        LCHK(launch_nt(NT, F_RECOVER_ADD, B * (N + 1) * w.rec_f(), B * (N + 1) * w.rec_b(), k_recover<S, E, true>,
                    Bi * (N + 1), s, pg, ws, out));
    }
    if (resid_out) {
        // after an adaptive sweep only the instances it touched changed
        if (p.fused) {
            LCHK(launch_nt(NT, F_RESID, B * (N + 1) * w.resid_f(), B * (N + 1) * w.resid_b(), k_resid_inst<S, E64, false>,
                        Bi, s, pg, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws, resid_out,
                        (int32_t*)nullptr, p.refine_tol));
        } else {
            LCHK(launch_nt(NT, F_RESID, B * (N + 1) * w.resid_f(), B * (N + 1) * w.resid_b(), k_resid<S, E64, false>,
                        Bi * (N + 1), s, pg, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws));
            LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, pg,
                        (const double*)dws, resid_out, (int32_t*)nullptr, p.refine_tol));
        }
    }
    return LQR_OK;
}

template <typename S, int TS>
int run_plain(const Plan& p, hipStream_t s, const In<S>& in, const Out<S>& out, S* ws, int32_t* iws,
              double* dws, double* resid_out) {
    using E = EngOf<S, TS>;
    using E64 = EngOf<double, TS>;
    constexpr int NT = E64::NT;
    const Work w(p, sizeof(S));
    const double B = (double)p.batch;
    const int64_t Bi = p.batch;
    LCHK(launch_nt(WG, F_CLEAR, 0, 4.0 * B, k_clear<int32_t>, (Bi + 255) / 256 * 4, s, out.status, Bi, iws,
                (int64_t)kQCount));
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
                    Bi * (p.N + 1), s, p, in, (const S*)out.x, (const S*)out.u, (const S*)out.lam, ws, dws));
        LCHK(launch_nt(WG, F_REDUCE, 0, B * 16.0 * (p.N + 1), k_resid_reduce<double>, (Bi + 63) / 64, s, p,
                    (const double*)dws, resid_out, (int32_t*)nullptr, p.refine_tol));
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
                (const double*)dws, rel, (int32_t*)nullptr, p.refine_tol));
    return LQR_OK;
}

#define LQR_RUNS(PREFIX, TSV)                                                                               \
    PREFIX template int run_scan<float, TSV>(const Plan&, hipStream_t, const In<float>&, const Out<float>&,  \
                                             float*, int32_t*, double*, int, double*, const Warm<float>&);  \
    PREFIX template int run_scan<double, TSV>(const Plan&, hipStream_t, const In<double>&, const Out<double>&,\
                                              double*, int32_t*, double*, int, double*, const Warm<double>&);\
    PREFIX template int run_plain<float, TSV>(const Plan&, hipStream_t, const In<float>&, const Out<float>&, \
                                              float*, int32_t*, double*, double*);                          \
    PREFIX template int run_plain<double, TSV>(const Plan&, hipStream_t, const In<double>&,                  \
                                               const Out<double>&, double*, int32_t*, double*, double*);     \
    PREFIX template int run_resid<float, TSV>(const Plan&, hipStream_t, const In<float>&, const float*,      \
                                              const float*, const float*, float*, double*, double*);        \
    PREFIX template int run_resid<double, TSV>(const Plan&, hipStream_t, const In<double>&, const double*,   \
                                               const double*, const double*, double*, double*, double*);

#define LQR_DECLARE_RUNS(TSV) LQR_RUNS(extern, TSV)
#define LQR_DEFINE_RUNS(TSV) LQR_RUNS(, TSV)

}  // namespace lqr
