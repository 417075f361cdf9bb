// bigeng.hpp -- workgroup-level dense linear algebra for blocks of order
// 65..256 (gfx950).
//
// One workgroup of four wavefronts (256 threads) owns one task.  Matrices of
// this size do not fit in registers or (several at a time) in LDS, so they
// live in global memory: the inputs and records, plus a per-workgroup
// scratch area for the intermediates of the task.  Every product is a
// workgroup GEMM on matrix cores: 64 x 64 output tiles, each wavefront a
// 32 x 32 quadrant of 2 x 2 MFMA 16x16x4 blocks, operands staged through LDS
// in k-chunks of 16.  Transposed operands are strided views, so no product
// copies a matrix.  Factorizations are blocked: a 32 x 32 diagonal block is
// factored and inverted in LDS by all 256 threads (one barrier per step),
// and the panel, trailing-update and inverse steps are GEMMs.
//
// Triangular solves are replaced by products with the explicit inverse of
// the Cholesky factor: every later step is then a matrix-core product.  The
// inverse of a Cholesky factor carries a relative error of order
// cond(L) * eps = sqrt(cond(P)) * eps, which the FP64-residual refinement
// removes; factors whose condition estimate exceeds the threshold are redone
// in FP64 anyway.
//
// Vectors use the "thread vector" layout: thread t holds element t (orders up
// to 256), the same contract as the lane vectors of the small-block engine,
// so the vector-only passes are shared between the two engines.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "engine.hpp"

namespace lqr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// MFMA 16x16x4: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator element r of lane l is D[row(l, r)][l % 16].  The FP32 and
// FP64 instructions order the four accumulator rows of a lane differently
// (measured on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using V = f32x4;
    static __device__ __forceinline__ V mac(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
    using V = f64x4;
    static __device__ __forceinline__ V mac(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// strided matrix view: element (i, j) at p[i * rs + j * cs]
// (orders <= 256: offsets fit in 32 bits)
template <typename P>
struct MV {
    P* p;
    int rs, cs;
    __device__ __forceinline__ P& operator()(int i, int j) const { return p[i * rs + j * cs]; }
    __device__ __forceinline__ MV<P> at(int i, int j) const { return MV<P>{&(*this)(i, j), rs, cs}; }
};
template <typename P> __device__ __forceinline__ MV<P> rowm(P* p, int ld) { return MV<P>{p, ld, 1}; }
template <typename P> __device__ __forceinline__ MV<P> trans(P* p, int ld) { return MV<P>{p, 1, ld}; }

// GEMM mode flags
enum : int {
    GM_LOWER = 1,   // compute and write only j <= i
    GM_SYM = 2,     // with GM_LOWER: also write out(j, i)
    GM_A_LO = 4,    // A(i, k) = 0 for k > i   (K range clipped per tile)
    GM_A_UP = 8,    // A(i, k) = 0 for k < i
    GM_B_LO = 16,   // B(k, j) = 0 for k < j
    GM_B_UP = 32,   // B(k, j) = 0 for k > j
    GM_ADD = 64,    // out = add + alpha * A B
    GM_IDENT = 128  // out += I
};

constexpr int BG_KC = 32;          // k-chunk staged in LDS
constexpr int BG_LDT = 64 + 16;    // LDS row stride of a staged chunk (bank spread of the 4 lane groups)

template <typename T>
struct BigLds {
    T vb[2][256];
    T As[BG_KC][BG_LDT];
    T Bs[BG_KC][BG_LDT];
    T D[32][33];    // diagonal block being factored (working copy)
    T F[32][33];    // its Cholesky factor
    T W[32][33];    // inverse being formed (working copy)
    T Fi[32][33];   // inverse of the factor
    double red[8];
    int flag[4];
};

template <typename T_>
struct BigEng {
    using T = T_;
    static constexpr bool BIG = true;
    static constexpr int NT = 256;   // threads per workgroup
    static constexpr int NP = 256;   // largest order
    static constexpr int GL = 256;
    int lg;
    __device__ explicit BigEng(int t) : lg(t) {}

    static __device__ __forceinline__ void sync() { __syncthreads(); }
    static __device__ __forceinline__ bool all(bool v) { return __syncthreads_and(v ? 1 : 0) != 0; }
    static __device__ __forceinline__ double sum(double v) {
        __shared__ double part[4];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
        __syncthreads();
        return part[0] + part[1] + part[2] + part[3];
    }

    // ------------------------------------------------------------ vectors
    template <typename S>
    __device__ __forceinline__ T vload(const S* g, int n) const { return lg < n ? T(g[lg]) : T(0); }
    template <typename S>
    __device__ __forceinline__ void vstore(S* g, int n, T v) const { if (lg < n) g[lg] = S(v); }

    // y = M x (TR: y = M' x) with M rows x cols (leading dim ld) in global
    // memory, x a thread vector; returns the thread vector y.  vb: LDS
    // staging of x (256 elements).
    template <bool TR, typename S>
    __device__ __forceinline__ T gmv(const S* M, int rows, int cols, int ld, T x, T* vb) const {
        stage_vec(vb, x);
        return gmv_v<TR>(M, rows, cols, ld, vb);
    }

    // stage a workgroup vector in vb (the interface of the wavefront
    // engine's staged products)
    __device__ __forceinline__ void stage_vec(T* vb, T x) const {
        __syncthreads();
        vb[lg] = x;
        __syncthreads();
    }

    // (the wavefront engine's prefetching form; here the same product)
    template <bool TR, bool WIDE = false, typename S>
    __device__ __forceinline__ T gmv_pf(const S* M, int rows, int cols, int ld, const T* vb) const {
        return gmv_v<TR>(M, rows, cols, ld, vb);
    }

    // gmv of a vector already staged in vb; the leading barrier keeps the
    // shared row results of the previous call until every thread read them
    template <bool TR, typename S>
    __device__ __forceinline__ T gmv_v(const S* M, int rows, int cols, int ld, const T* vb) const {
        __shared__ T yb[256];
        __syncthreads();
        if (TR) {
            T s = T(0);
            if (lg < cols) {
                const S* c = M + lg;
#pragma unroll 4
                for (int i = 0; i < rows; ++i) s = fma_(T(c[(int64_t)i * ld]), vb[i], s);
            }
            return s;
        }
        // one wavefront per row, lanes across the (contiguous) columns
        const int lane = lg & 63, wv = lg >> 6;
        for (int i = wv; i < rows; i += 4) {
            const S* r = M + (int64_t)i * ld;
            T s = T(0);
            for (int j = lane; j < cols; j += 64) s = fma_(T(r[j]), vb[j], s);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) yb[i] = s;
        }
        __syncthreads();
        return lg < rows ? yb[lg] : T(0);
    }

    // ------------------------------------------------------------- GEMM
    // out(i, j) = [add(i, j)] + [i == j] + alpha * sum_k A(i, k) B(k, j),
    // i < M, j < N, k < K.  Each output element is read (add) and written by
    // one thread after its tile's k-loop, so out may alias add, and may alias
    // A when every output tile reads only its own rows of A.  Ends with a
    // workgroup barrier (the result is visible to the whole workgroup).
    //
    // Software pipeline: while the matrix cores consume the k-chunk staged in
    // LDS, the global loads of the next chunk (of this tile, or the first
    // chunk of the next tile) are already in flight into registers.
    template <int F>
    __device__ __forceinline__ void tile_krange(int ti, int tj, int K, int& kb, int& ke) const {
        kb = 0;
        ke = K;
        if (F & GM_A_LO) ke = min(ke, (ti + 1) * 64);
        if (F & GM_A_UP) kb = max(kb, ti * 64);
        if (F & GM_B_LO) kb = max(kb, tj * 64);
        if (F & GM_B_UP) ke = min(ke, (tj + 1) * 64);
    }

    // next tile after (ti, tj) in row-major tile order (lower tiles only
    // with GM_LOWER); false when there is none
    template <int F>
    __device__ __forceinline__ bool next_tile(int& ti, int& tj, int nti, int ntj) const {
        ++tj;
        if (tj >= ntj || ((F & GM_LOWER) && tj > ti)) {
            tj = 0;
            ++ti;
        }
        return ti < nti;
    }

    template <typename PA, typename PB>
    __device__ __forceinline__ void load_chunk(T (&ra)[BG_KC / 4], T (&rb)[BG_KC / 4], const MV<PA>& A,
                                               const MV<PB>& B, int M, int N, int i0, int j0, int k0, int ke,
                                               bool a_kfast, bool b_jfast) const {
        const int t = lg;
#pragma unroll
        for (int r = 0; r < BG_KC / 4; ++r) {
            int i, kk;
            if (a_kfast) { kk = t % BG_KC; i = t / BG_KC + (256 / BG_KC) * r; }
            else { i = t & 63; kk = (t >> 6) + 4 * r; }
            ra[r] = (i0 + i < M && k0 + kk < ke) ? T(A(i0 + i, k0 + kk)) : T(0);
            int j, k2;
            if (b_jfast) { j = t & 63; k2 = (t >> 6) + 4 * r; }
            else { k2 = t % BG_KC; j = t / BG_KC + (256 / BG_KC) * r; }
            rb[r] = (j0 + j < N && k0 + k2 < ke) ? T(B(k0 + k2, j0 + j)) : T(0);
        }
    }

    __device__ __forceinline__ void store_chunk(BigLds<T>& L, const T (&ra)[BG_KC / 4], const T (&rb)[BG_KC / 4],
                                                bool a_kfast, bool b_jfast) const {
        const int t = lg;
#pragma unroll
        for (int r = 0; r < BG_KC / 4; ++r) {
            int i, kk;
            if (a_kfast) { kk = t % BG_KC; i = t / BG_KC + (256 / BG_KC) * r; }
            else { i = t & 63; kk = (t >> 6) + 4 * r; }
            L.As[kk][i] = ra[r];
            int j, k2;
            if (b_jfast) { j = t & 63; k2 = (t >> 6) + 4 * r; }
            else { k2 = t % BG_KC; j = t / BG_KC + (256 / BG_KC) * r; }
            L.Bs[k2][j] = rb[r];
        }
    }

    template <int F, typename PA, typename PB, typename PO, typename PC>
    __device__ __attribute__((noinline)) void gemm(BigLds<T>& L, int M, int N, int K, MV<PA> A, MV<PB> B,
                                                   MV<PO> out, MV<PC> add, T alpha = T(1)) const {
        using Mf = Mfma<T>;
        using V = typename Mf::V;
        static_assert(BG_KC % 16 == 0 && 64 * BG_KC == 256 * (BG_KC / 4), "chunk mapping");
        const int lane = lg & 63, wv = lg >> 6;
        const int wr = wv >> 1, wc = wv & 1;
        const int nti = (M + 63) >> 6, ntj = (N + 63) >> 6;
        const bool a_kfast = A.cs == 1, b_jfast = B.cs == 1;
        T ra[BG_KC / 4], rb[BG_KC / 4];
        bool have = false;   // registers hold the first chunk of the current tile
        int ti = 0, tj = 0;
        while (ti < nti) {
            int kb, ke;
            tile_krange<F>(ti, tj, K, kb, ke);
            const int i0 = ti * 64, j0 = tj * 64;
            if (!have && kb < ke) load_chunk(ra, rb, A, B, M, N, i0, j0, kb, ke, a_kfast, b_jfast);
            have = false;
            // the tile after this one (for the prefetch across tiles)
            int ni = ti, nj = tj;
            const bool more = next_tile<F>(ni, nj, nti, ntj);
            int nkb = 0, nke = 0;
            if (more) tile_krange<F>(ni, nj, K, nkb, nke);
            V acc[2][2];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = V{0, 0, 0, 0};
            for (int k0 = kb; k0 < ke; k0 += BG_KC) {
                __syncthreads();
                store_chunk(L, ra, rb, a_kfast, b_jfast);
                __syncthreads();
                if (k0 + BG_KC < ke) {
                    load_chunk(ra, rb, A, B, M, N, i0, j0, k0 + BG_KC, ke, a_kfast, b_jfast);
                } else if (more && nkb < nke) {
                    load_chunk(ra, rb, A, B, M, N, ni * 64, nj * 64, nkb, nke, a_kfast, b_jfast);
                    have = true;
                }
#pragma unroll
                for (int s = 0; s < BG_KC / 4; ++s) {
                    const int kr = 4 * s + (lane >> 4);
                    const T a0 = L.As[kr][wr * 32 + (lane & 15)];
                    const T a1 = L.As[kr][wr * 32 + 16 + (lane & 15)];
                    const T b0 = L.Bs[kr][wc * 32 + (lane & 15)];
                    const T b1 = L.Bs[kr][wc * 32 + 16 + (lane & 15)];
                    acc[0][0] = Mf::mac(a0, b0, acc[0][0]);
                    acc[0][1] = Mf::mac(a0, b1, acc[0][1]);
                    acc[1][0] = Mf::mac(a1, b0, acc[1][0]);
                    acc[1][1] = Mf::mac(a1, b1, acc[1][1]);
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = i0 + wr * 32 + a * 16 + Mf::row(lane, r);
                        const int j = j0 + wc * 32 + b * 16 + (lane & 15);
                        if (i >= M || j >= N) continue;
                        if ((F & GM_LOWER) && j > i) continue;
                        T v = alpha * acc[a][b][r];
                        if (F & GM_ADD) v += T(add(i, j));
                        if ((F & GM_IDENT) && i == j) v += T(1);
                        out(i, j) = (typename std::remove_cv<PO>::type)v;
                        if ((F & GM_SYM) && j < i) out(j, i) = (typename std::remove_cv<PO>::type)v;
                    }
            ti = ni;
            tj = nj;
            if (!more) break;
        }
        __syncthreads();
    }

    template <int F, typename PA, typename PB, typename PO>
    __device__ __forceinline__ void gemm(BigLds<T>& L, int M, int N, int K, MV<PA> A, MV<PB> B, MV<PO> out,
                                         T alpha = T(1)) const {
        static_assert(!(F & GM_ADD), "GM_ADD needs an add operand");
        gemm<F>(L, M, N, K, A, B, out, MV<const T>{nullptr, 0, 0}, alpha);
    }

    // elementwise copy of an n x n matrix (row-major, leading dims ldd, lds)
    template <typename D, typename S>
    __device__ __forceinline__ void copy(D* dst, int ldd, const S* src, int lds, int rows, int cols) const {
        for (int idx = lg; idx < rows * cols; idx += NT) {
            const int i = idx / cols, j = idx - i * cols;
            dst[(int64_t)i * ldd + j] = D(src[(int64_t)i * lds + j]);
        }
        __syncthreads();
    }

    // ------------------------------------------------- Cholesky + inverse
    // In place: the lower triangle of the n x n SPD matrix `a` (row-major,
    // leading dim n; the upper triangle is ignored on entry) becomes its
    // Cholesky factor L, with zeros above the diagonal; `li` (n x n) receives
    // L^{-1}, lower triangular with zeros above.  `tmp` holds 32 x n elements.
    // Returns (uniformly) whether every pivot was positive and finite, and
    // the extreme diagonal entries of L for the condition estimate.
    __device__ __forceinline__ bool potrf_inv(BigLds<T>& L, T* a, T* li, T* tmp, int n, T& dmin,
                                                        T& dmax) const {
        const int t = lg;
        bool ok = true;
        T mn = T(3.0e38), mx = T(0);
        const MV<T> A = rowm(a, n), Li = rowm(li, n);
        for (int kb = 0; kb < n; kb += 32) {
            const int w = min(32, n - kb);
            // diagonal block -> LDS (identity outside the logical size)
            for (int idx = t; idx < 32 * 32; idx += NT) {
                const int i = idx >> 5, j = idx & 31;
                T v = T(i == j ? 1 : 0);
                if (i < w && j < w && j <= i) v = A(kb + i, kb + j);
                L.D[i][j] = v;
                L.W[i][j] = T(i == j ? 1 : 0);
            }
            // right-looking factorization: step j reads column j of the
            // working copy, writes the final column j into F and updates the
            // trailing columns (distinct addresses, one barrier per step)
            for (int j = 0; j < 32; ++j) {
                __syncthreads();
                const T d = L.D[j][j];
                const T s = dsqrt(d);
                const T id = T(1) / d, is = T(1) / s;
                if (j < w) {
                    ok = ok && (d > T(0)) && finite_(d);
                    mn = s < mn ? s : mn;
                    mx = s > mx ? s : mx;
                }
                for (int idx = t; idx < 32 * 32; idx += NT) {
                    const int i = idx >> 5, c = idx & 31;
                    if (c == j && i >= j) L.F[i][j] = i == j ? s : L.D[i][j] * is;
                    else if (c > j && c <= i) L.D[i][c] -= L.D[i][j] * L.D[c][j] * id;
                }
            }
            __syncthreads();
            // inverse of the factor by forward elimination on the identity
            for (int j = 0; j < 32; ++j) {
                const T id = T(1) / L.F[j][j];
                for (int idx = t; idx < 32 * 32; idx += NT) {
                    const int i = idx >> 5, c = idx & 31;
                    if (c > j) continue;
                    if (i == j) L.Fi[j][c] = L.W[j][c] * id;
                    else if (i > j) L.W[i][c] -= L.F[i][j] * L.W[j][c] * id;
                }
                __syncthreads();
            }
            // write the diagonal blocks of L and L^{-1}; zero L right of the
            // block (the input's upper triangle) and L^{-1} right of the diagonal
            for (int idx = t; idx < w * n; idx += NT) {
                const int i = idx / n, j = idx - i * n;
                const int jj = j - kb;
                if (jj >= 0 && jj < w) {
                    A(kb + i, j) = jj <= i ? L.F[i][jj] : T(0);
                    Li(kb + i, j) = jj <= i ? L.Fi[i][jj] : T(0);
                } else if (jj >= w) {
                    A(kb + i, j) = T(0);
                    Li(kb + i, j) = T(0);
                }
            }
            __syncthreads();
            const int rest = n - kb - w;
            if (rest > 0) {
                // panel: L21 = A21 L11^{-T}
                gemm<0>(L, rest, w, w, A.at(kb + w, kb), MV<const T>{&Li(kb, kb), 1, n}, A.at(kb + w, kb));
                // trailing update (lower): A22 -= L21 L21'
                gemm<GM_LOWER | GM_ADD>(L, rest, rest, w, A.at(kb + w, kb), MV<const T>{&A(kb + w, kb), 1, n},
                                        A.at(kb + w, kb + w), MV<const T>{&A(kb + w, kb + w), n, 1}, T(-1));
            }
        }
        // off-diagonal blocks of L^{-1}, block row by block row:
        //   Li[r, 0:r] = -Li[r, r] (L[r, 0:r] Li[0:r, 0:r])
        const MV<T> Tm = rowm(tmp, n);
        for (int kb = 32; kb < n; kb += 32) {
            const int w = min(32, n - kb);
            gemm<GM_B_LO>(L, w, kb, kb, MV<const T>{&A(kb, 0), n, 1}, MV<const T>{li, n, 1}, Tm);
            gemm<GM_A_LO>(L, w, kb, w, MV<const T>{&Li(kb, kb), n, 1}, MV<const T>{tmp, n, 1}, Li.at(kb, 0), T(-1));
        }
        // uniform verdict and extremes (thread 0's view is every thread's)
        if (t == 0) {
            L.flag[0] = ok ? 1 : 0;
            L.red[0] = (double)mn;
            L.red[1] = (double)mx;
        }
        __syncthreads();
        const bool okall = L.flag[0] != 0;
        dmin = T(L.red[0]);
        dmax = T(L.red[1]);
        __syncthreads();
        return okall;
    }
};

}  // namespace lqr
