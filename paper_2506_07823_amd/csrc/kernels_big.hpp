// kernels_big.hpp -- matrix task bodies of the scan and plain paths for
// blocks of order 65..256 (BigEng: one 256-thread workgroup per task,
// products on matrix cores, intermediates in a per-workgroup scratch area).
//
// The steps and record layouts are those of the small-block bodies in
// kernels.hpp; only the arithmetic form differs: triangular solves with a
// Cholesky factor become products with its explicit inverse (computed by the
// blocked factorization), so every O(n^3) step is a matrix-core GEMM.
// Included by kernels.hpp after the shared helpers.
#pragma once

namespace lqr {

// scratch of the calling workgroup (elements of the compute type)
template <typename T, typename S>
__device__ __forceinline__ T* big_scratch(const Plan& p, S* ws) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + p.o_scr) + (int64_t)blockIdx.x * p.scr_elems;
}

template <typename P> __device__ __forceinline__ MV<const P> crm(const P* p, int ld) { return MV<const P>{p, ld, 1}; }
template <typename P> __device__ __forceinline__ MV<const P> ctr(const P* p, int ld) { return MV<const P>{p, 1, ld}; }

// ---------------------------------------------------------------------------
// Sec. II-D, eq. (initialization), as element_task:
//   R = L_R L_R',  W_B = L_R^{-1} B',  W_M = L_R^{-1} M',  w_r = L_R^{-1} r,
//   At = A - W_B' W_M,  Ct = W_B' W_B,  Pt = Q - W_M' W_M,
//   bt = c - W_B' w_r,  pt = q - W_M' w_r.
// ---------------------------------------------------------------------------
template <typename S, class E>
__device__ void big_element_task(BigLds<typename E::T>& L, const Plan& p, const In<S>& in, S* ws, int32_t* status, int64_t task) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = task / (N + 1);
    const int k = (int)(task % (N + 1));
    S* rec = ws + b * p.stride + p.o_tree + (int64_t)k * p.rec;
    const Ptr<S> P(p, in);
    if (k == N) {
        coop_zero(rec, 2 * nn);
        coop_copy(rec + 2 * nn, P.Q(b, N), nn);
        coop_zero(rec + 3 * nn, n);
        coop_copy(rec + 3 * nn + n, P.q(b, N), n);
        E::sync();
        return;
    }
    T* Lr = big_scratch<T>(p, ws);
    T* Lri = Lr + m * m;
    T* WB = Lri + m * m;
    T* WM = WB + m * n;
    T* tmp = WM + m * n;
    e.copy(Lr, m, P.R(b, k), m, m, m);
    T dmin, dmax;
    const bool ok = e.potrf_inv(L, Lr, Lri, tmp, m, dmin, dmax);
    fb_flag(p, ok, cond_est(dmin, dmax), b, status, 2);
    e.template gemm<GM_A_LO>(L, m, n, m, crm(Lri, m), ctr(P.B(b, k), m), rowm(WB, n));
    e.template gemm<GM_A_LO>(L, m, n, m, crm(Lri, m), ctr(P.M(b, k), m), rowm(WM, n));
    const T wr = e.template gmv<false>(Lri, m, m, m, e.vload(P.r(b, k), m), L.vb[0]);
    e.template gemm<GM_ADD>(L, n, n, m, ctr(WB, n), crm(WM, n), rowm(rec, n), crm(P.A(b, k), n), T(-1));
    e.template gemm<GM_LOWER | GM_SYM>(L, n, n, m, ctr(WB, n), crm(WB, n), rowm(rec + nn, n));
    e.template gemm<GM_LOWER | GM_SYM | GM_ADD>(L, n, n, m, ctr(WM, n), crm(WM, n), rowm(rec + 2 * nn, n),
                                                crm(P.Q(b, k), n), T(-1));
    const T bw = e.template gmv<true>(WB, m, n, n, wr, L.vb[1]);
    e.vstore(rec + 3 * nn, n, e.vload(P.c(b, k), n) - bw);
    const T pw = e.template gmv<true>(WM, m, n, n, wr, L.vb[0]);
    e.vstore(rec + 3 * nn + n, n, e.vload(P.q(b, k), n) - pw);
    E::sync();
}

// ---------------------------------------------------------------------------
// eq. (combination_rule), e1 (x) e2 (e1 earlier), as combine() in inverse
// form.  With P2 = L L', S = I + L' C1 L = L_S L_S', X = L_S^{-1} L':
//   Y = X A1,  Z1 = L^{-1} A2',  Z = L_S^{-1} Z1,
//   w1 = L_S^{-1}(L^{-1} p2 + L' b1),  w2 = X (b1 - C1 p2),
//   P = Y'Y + P1,  p = Y'w1 + p1,  A = Z'Y,  C = Z1'Z1 - Z'Z + C2,  b = Z'w2 + b2.
// CHEAP: e2 is a complete suffix, only P and p.
// ---------------------------------------------------------------------------
template <class E, bool CHEAP, typename S>
__device__ void big_combine(const E& e, BigLds<typename E::T>& L, typename E::T* scr, int n, const S* e1,
                            const S* P2, const S* p2v, const S* e2, S* outA, S* outC, S* outP, S* outb, S* outp,
                            bool& okp, typename E::T& kappa) {
    using T = typename E::T;
    const int nn = n * n;
    T* Lf = scr;
    T* Li = Lf + nn;
    T* W = Li + nn;
    T* Ls = W + nn;
    T* Lsi = Ls + nn;
    T* X = Lsi + nn;
    T* Y = X + nn;
    T* Z1 = Y + nn;
    T* tmp = Z1 + nn;
    const S* A1 = e1;
    const S* C1 = e1 + nn;
    const S* P1 = e1 + 2 * nn;
    const S* b1 = e1 + 3 * nn;
    const S* p1 = e1 + 3 * nn + n;
    e.copy(Lf, n, P2, n, n, n);
    T dmin, dmax;
    bool ok = e.potrf_inv(L, Lf, Li, tmp, n, dmin, dmax);
    T kap = cond_est(dmin, dmax);
    e.template gemm<GM_B_LO>(L, n, n, n, crm(C1, n), crm(Lf, n), rowm(W, n));                     // W = C1 L
    e.template gemm<GM_LOWER | GM_IDENT | GM_A_UP>(L, n, n, n, ctr(Lf, n), crm(W, n), rowm(Ls, n));  // I + L'W
    ok = e.potrf_inv(L, Ls, Lsi, tmp, n, dmin, dmax) && ok;
    {
        const T ks = cond_est(dmin, dmax);
        kap = ks > kap ? ks : kap;
    }
    e.template gemm<GM_A_LO | GM_B_UP>(L, n, n, n, crm(Lsi, n), ctr(Lf, n), rowm(X, n));         // X = L_S^{-1} L'
    e.template gemm<0>(L, n, n, n, crm(X, n), crm(A1, n), rowm(Y, n));                            // Y = X A1
    e.template gemm<GM_LOWER | GM_SYM | GM_ADD>(L, n, n, n, ctr(Y, n), crm(Y, n), rowm(outP, n), crm(P1, n));
    const T p2 = e.vload(p2v, n);
    const T g = e.template gmv<false>(Li, n, n, n, p2, L.vb[0]);
    const T lb = e.template gmv<true>(Lf, n, n, n, e.vload(b1, n), L.vb[1]);
    const T w1 = e.template gmv<false>(Lsi, n, n, n, g + lb, L.vb[0]);
    const T pv = e.template gmv<true>(Y, n, n, n, w1, L.vb[1]) + e.vload(p1, n);
    e.vstore(outp, n, pv);
    if (!CHEAP) {
        const S* A2 = e2;
        const S* C2 = e2 + nn;
        const S* b2 = e2 + 3 * nn;
        e.template gemm<GM_A_LO>(L, n, n, n, crm(Li, n), ctr(A2, n), rowm(Z1, n));     // Z1 = L^{-1} A2'
        e.template gemm<GM_A_LO>(L, n, n, n, crm(Lsi, n), crm(Z1, n), rowm(W, n));     // Z = L_S^{-1} Z1
        e.template gemm<0>(L, n, n, n, ctr(W, n), crm(Y, n), rowm(outA, n));           // A = Z'Y
        e.template gemm<GM_LOWER | GM_ADD>(L, n, n, n, ctr(Z1, n), crm(Z1, n), rowm(Ls, n), crm(C2, n));
        e.template gemm<GM_LOWER | GM_SYM | GM_ADD>(L, n, n, n, ctr(W, n), crm(W, n), rowm(outC, n), crm(Ls, n),
                                                    T(-1));
        const T cp = e.template gmv<false>(C1, n, n, n, p2, L.vb[0]);
        const T w2 = e.template gmv<false>(X, n, n, n, e.vload(b1, n) - cp, L.vb[1]);
        const T bv = e.template gmv<true>(W, n, n, n, w2, L.vb[0]) + e.vload(b2, n);
        e.vstore(outb, n, bv);
    }
    E::sync();
    okp = ok;
    kappa = kap;
}

template <typename S, class E>
__device__ void big_up_task(BigLds<typename E::T>& L, const Plan& p, S* ws, int lvl, int32_t* status,
                            int64_t task) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int n = p.n, nn = n * n;
    const int cout = p.rt.cnt[lvl + 1], cin = p.rt.cnt[lvl];
    const int64_t b = task / cout;
    const int i = (int)(task % cout);
    S* base = ws + b * p.stride + p.o_tree;
    const S* e1 = base + (int64_t)(p.rt.off[lvl] + 2 * i) * p.rec;
    S* out = base + (int64_t)(p.rt.off[lvl + 1] + i) * p.rec;
    if (2 * i + 1 >= cin) {
        coop_copy(out, e1, p.rec);
        E::sync();
        return;
    }
    const S* e2 = e1 + p.rec;
    bool ok;
    T kappa;
    big_combine<E, false>(e, L, big_scratch<T>(p, ws), n, e1, e2 + 2 * nn, e2 + 3 * nn + n, e2, out, out + nn,
                          out + 2 * nn, out + 3 * nn, out + 3 * nn + n, ok, kappa);
    fb_flag(p, ok, kappa, b, status, 4);
}

template <typename S, class E>
__device__ void big_down_task(BigLds<typename E::T>& L, const Plan& p, S* ws, int lvl, int32_t* status,
                              int64_t task) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int n = p.n, nn = n * n;
    const int half = p.rt.cnt[lvl] / 2;
    const int64_t b = task / half;
    const int j = 2 * (int)(task % half) + 1;
    S* tree = ws + b * p.stride + p.o_tree;
    S* suf = ws + b * p.stride + p.o_suf;
    const S* node = tree + (int64_t)(p.rt.off[lvl] + j) * p.rec;
    S* out = suf + (int64_t)(p.rt.off[lvl] + j) * p.srec;
    const int i1 = (j + 1) / 2;
    if (i1 >= p.rt.cnt[lvl + 1]) {
        coop_copy(out, node + 2 * nn, nn);
        coop_copy(out + nn, node + 3 * nn + n, n);
        E::sync();
        return;
    }
    const S* s2 = suf + (int64_t)suffix_id(p.rt, lvl + 1, i1) * p.srec;
    bool ok;
    T kappa;
    big_combine<E, true>(e, L, big_scratch<T>(p, ws), n, node, s2, s2 + nn, (const S*)nullptr, (S*)nullptr,
                         (S*)nullptr, out, (S*)nullptr, out + nn, ok, kappa);
    fb_flag(p, ok, kappa, b, status, 4);
}

// ---------------------------------------------------------------------------
// eq. (lqr) per stage and eq. (controlled_dynamics), as policy_task.  The
// refinement needs G^{-1} = L_G^{-T} L_G^{-1}: the record keeps L_G^{-1}.
// ---------------------------------------------------------------------------
template <typename S, class E>
__device__ void big_policy_task(BigLds<typename E::T>& L, const Plan& p, const In<S>& in, S* ws, int32_t* status, int64_t task) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const int64_t b = task / N;
    const int k = (int)(task % N);
    const Ptr<S> P(p, in);
    S* inst = ws + b * p.stride;
    const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
    T* T1 = big_scratch<T>(p, ws);
    T* G = T1 + n * m;
    T* Gi = G + m * m;
    T* H = Gi + m * m;
    T* H2 = H + m * n;
    T* KT = H2 + m * n;
    T* tmp = KT + m * n;
    e.template gemm<0>(L, n, m, n, crm(Pn, n), crm(P.B(b, k), m), rowm(T1, m));                        // P'B
    e.template gemm<GM_LOWER | GM_ADD>(L, m, m, n, ctr(P.B(b, k), m), crm(T1, m), rowm(G, m), crm(P.R(b, k), m));
    e.template gemm<GM_ADD>(L, m, n, n, ctr(T1, m), crm(P.A(b, k), n), rowm(H, n), ctr(P.M(b, k), m));  // M' + (P'B)'A
    const T v = e.template gmv<false>(Pn, n, n, n, e.vload(P.c(b, k), n), L.vb[0]) + e.vload(Pn + nn, n);
    const T h = e.template gmv<true>(P.B(b, k), n, m, m, v, L.vb[1]) + e.vload(P.r(b, k), m);
    T dmin, dmax;
    const bool ok = e.potrf_inv(L, G, Gi, tmp, m, dmin, dmax);
    fb_flag(p, ok, cond_est(dmin, dmax), b, status, 2);
    e.template gemm<GM_A_LO>(L, m, n, m, crm(Gi, m), crm(H, n), rowm(H2, n));                   // L_G^{-1} H
    e.template gemm<GM_A_UP>(L, m, n, m, ctr(Gi, m), crm(H2, n), rowm(KT, n), T(-1));            // K = -G^{-1} H
    const T t = e.template gmv<false>(Gi, m, m, m, h, L.vb[0]);
    const T kf = -e.template gmv<true>(Gi, m, m, m, t, L.vb[1]);
    e.copy(inst + p.o_K + (int64_t)k * m * n, n, KT, n, m, n);
    e.vstore(inst + p.o_kff + (int64_t)k * m, m, kf);
    e.copy(inst + p.o_LG + (int64_t)k * m * m, m, Gi, m, m, m);
    S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
    e.template gemm<GM_ADD>(L, n, n, m, crm(P.B(b, k), m), crm(KT, n), rowm(leaf, n), crm(P.A(b, k), n));  // A + B K
    const T bb = e.template gmv<false>(P.B(b, k), n, m, m, kf, L.vb[0]) + e.vload(P.c(b, k), n);
    e.vstore(leaf + nn, n, bb);
    E::sync();
}

// forward tree up-sweep, matrix part: M = M_r M_l, v = M_r v_l + v_r
template <typename S, class E>
__device__ void big_fup_task(BigLds<typename E::T>& L, const S* l, const S* r, S* out, int n) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int nn = n * n;
    e.template gemm<0>(L, n, n, n, crm(r, n), crm(l, n), rowm(out, n));
    const T v = e.template gmv<false>(r, n, n, n, e.vload(l + nn, n), L.vb[0]) + e.vload(r + nn, n);
    e.vstore(out + nn, n, v);
    E::sync();
}

// refinement, per stage: kff'_k = -G^{-1} h'_k with the stored L_G^{-1}
template <typename S, class E, class LT>
__device__ void big_ref_kff(LT& L, const Plan& p, const In<S>& in, S* ws, int64_t b, int k) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int n = p.n, m = p.m, nn = n * n;
    const Ptr<S> P(p, in);
    S* inst = ws + b * p.stride;
    const S* Pn = inst + p.o_suf + (int64_t)suffix_id(p.rt, 0, k + 1) * p.srec;
    const S* leaf = inst + p.o_ftree + (int64_t)k * p.frec;
    const S* Gi = inst + p.o_LG + (int64_t)k * m * m;
    const T pn = e.vload(inst + p.o_pend + (int64_t)k * n, n);
    const T cpv = e.vload(inst + p.o_cp + (int64_t)k * n, n);
    const T v = pn + e.template gmv<false>(Pn, n, n, n, cpv, L.vb[0]);
    const T pk = e.template gmv<true>(leaf, n, n, n, pn, L.vb[1]) + e.vload(inst + p.o_w + (int64_t)k * n, n);
    e.vstore(inst + p.o_pp + (int64_t)k * n, n, pk);
    const T h = e.template gmv<true>(P.B(b, k), n, m, m, v, L.vb[0]) + e.vload(inst + p.o_rp + (int64_t)k * m, m);
    const T t = e.template gmv<false>(Gi, m, m, m, h, L.vb[1]);
    const T kf = -e.template gmv<true>(Gi, m, m, m, t, L.vb[0]);
    e.vstore(inst + p.o_kffp + (int64_t)k * m, m, kf);
    const T bb = e.template gmv<false>(P.B(b, k), n, m, m, kf, L.vb[1]) + cpv;
    e.vstore(inst + p.o_ftree + (int64_t)k * p.frec + nn, n, bb);
    E::sync();
}

// ---------------------------------------------------------------------------
// Plain baseline for large blocks: the sequential Riccati recursion of
// eq. (lqr) for instance b.  Inputs and outputs of type S; P_k, p_k, K_k, k_k
// in `inst` of type W, the intermediates of one step in `scr` (compute type).
// ---------------------------------------------------------------------------
template <typename S, typename W, class E>
__device__ void big_plain_body(BigLds<typename E::T>& L, const Plan& p, const In<S>& in, const Out<S>& out, W* inst,
                               typename E::T* scr, int64_t b) {
    using T = typename E::T;
    const E e(threadIdx.x);
    const int N = p.N, n = p.n, m = p.m, nn = n * n;
    const Ptr<S> P(p, in);
    T* Pc = scr;
    T* PA = Pc + nn;
    T* T1 = PA + nn;
    T* G = T1 + n * m;
    T* Gi = G + m * m;
    T* H = Gi + m * m;
    T* H2 = H + m * n;
    T* KT = H2 + m * n;
    T* tmp = KT + m * n;
    W* Pst = inst + p.o_suf;
    e.copy(Pc, n, P.Q(b, N), n, n, n);
    e.copy(Pst + (int64_t)N * p.srec, n, Pc, n, n, n);
    T pn = e.vload(P.q(b, N), n);
    e.vstore(Pst + (int64_t)N * p.srec + nn, n, pn);
    bool ok = true;
    for (int k = N - 1; k >= 0; --k) {
        e.template gemm<0>(L, n, m, n, crm(Pc, n), crm(P.B(b, k), m), rowm(T1, m));
        e.template gemm<GM_LOWER | GM_ADD>(L, m, m, n, ctr(P.B(b, k), m), crm(T1, m), rowm(G, m),
                                           crm(P.R(b, k), m));
        e.template gemm<GM_ADD>(L, m, n, n, ctr(T1, m), crm(P.A(b, k), n), rowm(H, n), ctr(P.M(b, k), m));
        e.template gemm<0>(L, n, n, n, crm(Pc, n), crm(P.A(b, k), n), rowm(PA, n));
        const T v = e.template gmv<false>(Pc, n, n, n, e.vload(P.c(b, k), n), L.vb[0]) + pn;
        const T h = e.template gmv<true>(P.B(b, k), n, m, m, v, L.vb[1]) + e.vload(P.r(b, k), m);
        const T pa = e.template gmv<true>(P.A(b, k), n, n, n, v, L.vb[0]);
        T dmin, dmax;
        ok = e.potrf_inv(L, G, Gi, tmp, m, dmin, dmax) && ok;
        e.template gemm<GM_A_LO>(L, m, n, m, crm(Gi, m), crm(H, n), rowm(H2, n));
        e.template gemm<GM_A_UP>(L, m, n, m, ctr(Gi, m), crm(H2, n), rowm(KT, n), T(-1));
        const T t = e.template gmv<false>(Gi, m, m, m, h, L.vb[1]);
        const T kf = -e.template gmv<true>(Gi, m, m, m, t, L.vb[0]);
        e.copy(inst + p.o_K + (int64_t)k * m * n, n, KT, n, m, n);
        e.vstore(inst + p.o_kff + (int64_t)k * m, m, kf);
        // P_k = Q + A'(P'A) + K'H,  p_k = q + A'v + K'h
        e.template gemm<GM_LOWER | GM_SYM | GM_ADD>(L, n, n, n, ctr(P.A(b, k), n), crm(PA, n), rowm(Pc, n),
                                                    crm(P.Q(b, k), n));
        e.template gemm<GM_LOWER | GM_SYM | GM_ADD>(L, n, n, m, ctr(KT, n), crm(H, n), rowm(Pc, n), crm(Pc, n));
        pn = e.vload(P.q(b, k), n) + pa + e.template gmv<true>(KT, m, n, n, h, L.vb[1]);
        e.copy(Pst + (int64_t)k * p.srec, n, Pc, n, n, n);
        e.vstore(Pst + (int64_t)k * p.srec + nn, n, pn);
    }
    if (!ok) set_status(out.status, b, 2);
    // forward pass and costates
    T x = e.vload(P.x0(b), n);
    bool fin = true;
    for (int k = 0; k <= N; ++k) {
        const W* Pk = Pst + (int64_t)k * p.srec;
        const T lam = e.template gmv<false>(Pk, n, n, n, x, L.vb[0]) + e.vload(Pk + nn, n);
        e.vstore(out.x + (b * (N + 1) + k) * n, n, x);
        e.vstore(out.lam + (b * (N + 1) + k) * n, n, lam);
        fin = fin && (e.lg >= n || (finite_(x) && finite_(lam)));
        if (k == N) break;
        const T u = e.template gmv<false>(inst + p.o_K + (int64_t)k * m * n, m, n, n, x, L.vb[1]) +
                    e.vload(inst + p.o_kff + (int64_t)k * m, m);
        e.vstore(out.u + (b * N + k) * m, m, u);
        fin = fin && (e.lg >= m || finite_(u));
        const T xa = e.template gmv<false>(P.A(b, k), n, n, n, x, L.vb[0]);
        const T xb = e.template gmv<false>(P.B(b, k), n, m, m, u, L.vb[1]);
        x = xa + xb + e.vload(P.c(b, k), n);
    }
    if (!E::all(fin)) set_status(out.status, b, 1);
    E::sync();
}

// one workgroup per instance (grid-stride over the instances)
template <typename S, class E>
__global__ __launch_bounds__(256) void k_plain_big(Plan p, In<S> in, Out<S> out, S* ws) {
    using T = typename E::T;
    __shared__ BigLds<T> L;
    for (int64_t b = blockIdx.x; b < p.batch; b += gridDim.x)
        big_plain_body<S, S, E>(L, p, in, out, ws + b * p.stride, big_scratch<T>(p, ws), b);
}

// FP64 redo of marked instances (as k_redo), large blocks: FP64 slot and
// FP64 scratch of the calling workgroup
template <typename S, class E64>
__global__ __launch_bounds__(256) void k_redo_big(Plan rp, In<S> in, Out<S> out, double* ws64) {
    __shared__ BigLds<double> L;
    for (int64_t b = blockIdx.x; b < rp.batch; b += gridDim.x) {
        if (!(out.status[b] & 8)) continue;   // uniform across the workgroup
        __syncthreads();
        if (threadIdx.x == 0) out.status[b] = 8;
        __syncthreads();
        big_plain_body<S, double, E64>(L, rp, in, out, ws64 + (int64_t)blockIdx.x * rp.stride,
                                       big_scratch<double>(rp, ws64), b);
    }
}

}  // namespace lqr
