// engine.hpp -- wavefront-level dense linear algebra on small blocks (gfx950).
//
// One *group* of G x G lanes of a 64-wide wavefront owns one task (one scan
// combine, one stage, ...).  A G=8 group is a whole wavefront; G=4 packs four
// independent tasks into one wavefront.  Working matrices of padded order
// NP = G*TS live in registers as TS x TS tiles: lane (ty, tx) owns the
// entries (ty + G*a, tx + G*b), a, b < TS.  Matrices that other lanes must
// read (the right-hand operands of a product, triangular factors) are staged
// in the group's LDS slots with an odd leading dimension LD = NP + 1, so
// that the strided row/column reads of one k-step fall into distinct banks.
// Every matrix keeps zeros outside its logical size, which lets products run
// over the padded tile without masks.
//
// Vectors use the "lane vector" layout: lane lg (0 <= lg < G*G) of the group
// holds element lg (NP <= G*G is required).
//
// Sequential chains (Cholesky, triangular solves) run right-looking: at step
// k the owners of column (row) k publish it through a small LDS buffer and
// every lane updates its own tile entries, so the chain costs one
// workgroup barrier per step and the update work is spread over all lanes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lqr {

template <typename T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_sqrtf(x); }
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return __builtin_sqrt(x); }

// Pivot of a Cholesky step (d > 0): s = sqrt(d) and inv = 1 / s.  FP32: the
// hardware reciprocal square root (about 1 ulp) and one product, two
// instructions on the factorization's dependent chain where the correctly
// rounded square root and division take about 25 (the FP32 solution is
// refined against an FP64 residual).  The hardware operation reads a
// subnormal input as zero, so a pivot below the smallest normal number is
// scaled by 2^32 first (exact) and the result by 2^16, since
// rsq(2^32 d) = 2^-16 rsq(d): selects, no branch.  FP64: correctly rounded.
__device__ __forceinline__ void pivot_root(float d, float& s, float& inv) {
    const bool tiny = d < 1.17549435e-38f;
    const float r = __builtin_amdgcn_rsqf(tiny ? d * 4294967296.0f : d);
    inv = tiny ? r * 65536.0f : r;
    s = d * inv;
}
__device__ __forceinline__ void pivot_root(double d, double& s, double& inv) {
    s = __builtin_sqrt(d);
    inv = 1.0 / s;
}

// Every kernel of this library runs workgroups of exactly one wavefront, so
// lanes hand data to each other through LDS with a wavefront-scope fence:
// LDS instructions of one wavefront execute in issue order, and the fence
// keeps the compiler from moving LDS accesses across the hand-off (a
// workgroup barrier would also drain every outstanding global load).
// fused multiply-add in the operands' own precision (the unsuffixed builtin
// is the double one and would promote float operands)
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Value of v in lane k, k uniform across the wavefront (a scalar read of
// one lane's register: no LDS traffic).
__device__ __forceinline__ float lane_at(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double lane_at(double v, int k) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), k),
                            __builtin_amdgcn_readlane(__double2loint(v), k));
}

template <typename T>
__device__ __forceinline__ bool finite_(T v) { return __builtin_isfinite(v); }

__device__ __forceinline__ bool wave_all(bool v) {
    return __builtin_amdgcn_ballot_w64(!v) == 0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ void wg_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T_, int G_, int TS_>
struct Eng {
    using T = T_;
    static constexpr int G = G_;
    static constexpr int TS = TS_;
    static constexpr int NP = G * TS;        // padded order
    static constexpr int LD = NP + 1;        // LDS leading dimension
    static constexpr int MAT = NP * LD;      // LDS elements per matrix slot
    static constexpr int GL = G * G;         // lanes per group
    static_assert(NP <= GL, "lane-vector layout needs NP <= G*G");
    static_assert(64 % GL == 0, "groups must tile a wavefront");
    static constexpr bool BIG = false;
    static constexpr int NT = 64;   // threads per workgroup

    static __device__ __forceinline__ void sync() { wg_sync(); }
    static __device__ __forceinline__ bool all(bool v) { return wave_all(v); }
    static __device__ __forceinline__ double sum(double v) { return wave_sum(v); }

    int lg, ty, tx;
    __device__ explicit Eng(int lane_in_group)
        : lg(lane_in_group), ty(lane_in_group / G), tx(lane_in_group % G) {}

    __device__ __forceinline__ int row(int a) const { return ty + G * a; }
    __device__ __forceinline__ int col(int b) const { return tx + G * b; }

    using Tile = T[TS][TS];

    // ---------------------------------------------------------------- tiles
    __device__ __forceinline__ static void zero(Tile& t) {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) t[a][b] = T(0);
    }

    // t = G[rows x cols] (row-major, leading dim ldg), or its transpose when
    // TR (then G is cols x rows and t = G'); zero outside.
    template <bool TR = false, typename S>
    __device__ __forceinline__ void load(Tile& t, const S* g, int rows, int cols, int ldg) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) {
                const int i = row(a), j = col(b);
                T v = T(0);
                if (i < rows && j < cols) v = T(TR ? g[(int64_t)j * ldg + i] : g[(int64_t)i * ldg + j]);
                t[a][b] = v;
            }
    }

    // t += G (same conventions)
    template <bool TR = false, typename S>
    __device__ __forceinline__ void add_global(Tile& t, const S* g, int rows, int cols, int ldg, T scale = T(1)) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) {
                const int i = row(a), j = col(b);
                if (i < rows && j < cols)
                    t[a][b] += scale * T(TR ? g[(int64_t)j * ldg + i] : g[(int64_t)i * ldg + j]);
            }
    }

    template <typename S>
    __device__ __forceinline__ void store(const Tile& t, S* g, int rows, int cols, int ldg) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) {
                const int i = row(a), j = col(b);
                if (i < rows && j < cols) g[(int64_t)i * ldg + j] = S(t[a][b]);
            }
    }

    // store the lower triangle of t mirrored into both triangles of g (n x n):
    // the output is exactly symmetric.
    template <typename S>
    __device__ __forceinline__ void store_sym(const Tile& t, S* g, int n) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) {
                const int i = row(a), j = col(b);
                if (i < n && j <= i) {
                    g[(int64_t)i * n + j] = S(t[a][b]);
                    if (j < i) g[(int64_t)j * n + i] = S(t[a][b]);
                }
            }
    }

    __device__ __forceinline__ void to_lds(const Tile& t, T* s) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) s[row(a) * LD + col(b)] = t[a][b];
    }

    // the first RB row blocks of t (rows < G * RB) to an LDS region
    template <int RB>
    __device__ __forceinline__ void to_lds_rows(const Tile& t, T* s) const {
        static_assert(RB <= TS, "block limit");
#pragma unroll
        for (int a = 0; a < RB; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) s[row(a) * LD + col(b)] = t[a][b];
    }

    __device__ __forceinline__ void from_lds(Tile& t, const T* s) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) t[a][b] = s[row(a) * LD + col(b)];
    }

    __device__ __forceinline__ void add_identity(Tile& t, int n, T s = T(1)) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b)
                if (row(a) == col(b) && row(a) < n) t[a][b] += s;
    }

    // acc (+)= op(X) op(Y) over k < K, X and Y in LDS slots.
    // op(X)(i,k) = TX ? X[k][i] : X[i][k];  op(Y)(k,j) = TY ? Y[j][k] : Y[k][j].
    // SYM: the product is symmetric and only its lower triangle is needed;
    // the strictly-upper tile blocks (b > a) are skipped.  SUB: subtract.
    // RA / CB: only the first RA row blocks and CB column blocks of the tile
    // are formed (products whose result has fewer than NP rows or columns).
    template <bool TX, bool TY, bool SYM = false, bool SUB = false, int RA = TS, int CB = TS>
    __device__ __forceinline__ void gemm(Tile& acc, const T* X, const T* Y, int K) const {
        static_assert(RA <= TS && CB <= TS, "block limits");
#pragma unroll 2
        for (int k = 0; k < K; ++k) {
            T xa[RA], yb[CB];
#pragma unroll
            for (int a = 0; a < RA; ++a) xa[a] = TX ? X[k * LD + row(a)] : X[row(a) * LD + k];
#pragma unroll
            for (int b = 0; b < CB; ++b) yb[b] = TY ? Y[col(b) * LD + k] : Y[k * LD + col(b)];
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < CB; ++b)
                    if (!SYM || b <= a) acc[a][b] = fma_(SUB ? -xa[a] : xa[a], yb[b], acc[a][b]);
        }
    }

    template <bool TX, bool TY, bool SYM = false, int RA = TS, int CB = TS>
    __device__ __forceinline__ void gemm_sub(Tile& acc, const T* X, const T* Y, int K) const {
        gemm<TX, TY, SYM, true, RA, CB>(acc, X, Y, K);
    }

    // gemm with a triangular factor: TRI = 1 when Y is lower triangular
    // (Y(k, c) = 0 for c > k), TRI = 2 when op(X) is upper triangular
    // (X(r, k) = 0 for r > k, e.g. the transpose of a lower factor).  The
    // k loop runs in segments of G (one block row), and segment j skips the
    // column blocks b > j (TRI 1) or row blocks a > j (TRI 2), whose
    // products are exact zeros there: about 40 % fewer FMAs and LDS reads.
    template <bool TX, bool TY, bool SYM, int TRI>
    __device__ __forceinline__ void gemm_tri(Tile& acc, const T* X, const T* Y, int K) const {
        static_assert(TRI == 1 || TRI == 2, "triangular operand");
#pragma unroll
        for (int j = 0; j < TS; ++j) {
            const int k0 = G * j;
            if (k0 >= K) break;
            const int k1 = k0 + G < K ? k0 + G : K;
#pragma unroll 2
            for (int k = k0; k < k1; ++k) {
                T xa[TS], yb[TS];
#pragma unroll
                for (int a = 0; a < TS; ++a)
                    if (TRI != 2 || a <= j) xa[a] = TX ? X[k * LD + row(a)] : X[row(a) * LD + k];
#pragma unroll
                for (int b = 0; b < TS; ++b)
                    if (TRI != 1 || b <= j) yb[b] = TY ? Y[col(b) * LD + k] : Y[k * LD + col(b)];
#pragma unroll
                for (int a = 0; a < TS; ++a)
#pragma unroll
                    for (int b = 0; b < TS; ++b)
                        if ((!SYM || b <= a) && (TRI != 1 || b <= j) && (TRI != 2 || a <= j))
                            acc[a][b] = fma_(xa[a], yb[b], acc[a][b]);
            }
        }
    }

    // -------------------------------------------- coalesced global <-> LDS
    // Whole-slot copy of a rows x cols global matrix (leading dim ldg) into an
    // LDS slot, zero outside: consecutive lanes read consecutive elements.
    template <typename S>
    __device__ __forceinline__ void g2s(T* slot, const S* g, int rows, int cols, int ldg) const {
        for (int idx = lg; idx < NP * NP; idx += GL) {
            const int i = idx / NP, j = idx - (idx / NP) * NP;
            slot[i * LD + j] = (i < rows && j < cols) ? T(g[(int64_t)i * ldg + j]) : T(0);
        }
    }

    // g2s for the dependent chains of the combine: each lane copies
    // NP^2 / GL elements (NP is a multiple of 8, so that is exact) in groups
    // of G2S_U whose loads are all issued before the group's stores, one
    // wait per group instead of one per element (more registers in flight)
    static constexpr int G2S_IT = NP * NP / GL;
    static constexpr int G2S_U = G2S_IT % 8 == 0 ? 8 : G2S_IT % 5 == 0 ? 5 : G2S_IT % 4 == 0 ? 4
                               : G2S_IT % 3 == 0 ? 3 : G2S_IT % 2 == 0 ? 2 : 1;
    template <typename S>
    __device__ __forceinline__ void g2s_batched(T* slot, const S* g, int rows, int cols, int ldg) const {
        static_assert(G2S_IT * GL == NP * NP, "whole slot in equal lane shares");
#pragma unroll 1
        for (int it0 = 0; it0 < G2S_IT; it0 += G2S_U) {
            T v[G2S_U];
#pragma unroll
            for (int u = 0; u < G2S_U; ++u) {
                const int idx = lg + (it0 + u) * GL;
                const int i = idx / NP, j = idx - (idx / NP) * NP;
                // 32-bit offset from the uniform base (a slot's matrix is at
                // most 256 x 256)
                v[u] = (i < rows && j < cols) ? T(g[i * ldg + j]) : T(0);
            }
#pragma unroll
            for (int u = 0; u < G2S_U; ++u) {
                const int idx = lg + (it0 + u) * GL;
                const int i = idx / NP, j = idx - (idx / NP) * NP;
                slot[i * LD + j] = v[u];
            }
        }
    }
    // rows x cols of an LDS slot to global memory (coalesced)
    template <typename S>
    __device__ __forceinline__ void s2g(const T* slot, S* g, int rows, int cols, int ldg) const {
        const float inv = 1.0f / (float)cols;
        for (int idx = lg; idx < rows * cols; idx += GL) {
            const int i = (int)(((float)idx + 0.5f) * inv);
            const int j = idx - i * cols;
            g[(int64_t)i * ldg + j] = S(slot[i * LD + j]);
        }
    }
    // tile <- slot transposed
    __device__ __forceinline__ void from_lds_t(Tile& t, const T* s) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b < TS; ++b) t[a][b] = s[col(b) * LD + row(a)];
    }
    // lower triangle of t mirrored into both triangles of an LDS slot
    __device__ __forceinline__ void to_lds_sym(const Tile& t, T* s) const {
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                const int i = row(a), j = col(b);
                if (j <= i) {
                    s[i * LD + j] = t[a][b];
                    s[j * LD + i] = t[a][b];
                }
            }
    }

    // ------------------------------------------------------- lane vectors
    template <typename S>
    __device__ __forceinline__ T vload(const S* g, int n) const { return lg < n ? T(g[lg]) : T(0); }
    template <typename S>
    __device__ __forceinline__ void vstore(S* g, int n, T v) const { if (lg < n) g[lg] = S(v); }

    // y = op(X) v over k < K for rows < rows (X in LDS; v staged through vb).
    // The workgroup is one wavefront, whose LDS accesses complete in
    // program order, so successive calls may share one vb.
    template <bool TX>
    __device__ __forceinline__ T matvec(const T* X, T* vb, T v, int K, int rows) const {
        if (lg < NP) vb[lg] = v;
        wg_sync();
        T s = T(0);
        if (lg < rows) {
            // unrolled so that several LDS reads are in flight per wait (the
            // accumulation order is unchanged)
#pragma unroll 4
            for (int k = 0; k < K; ++k)
                s = fma_(TX ? X[k * LD + lg] : X[lg * LD + k], vb[k], s);
        }
        return s;
    }

    // y = op(M) x straight from global memory (no staging of M): M is a
    // rows x cols matrix with leading dim ld; x is a lane vector of length
    // (TR ? rows : cols) staged through vb.  TR: y = M' x (length cols), lane j
    // reads column j, coalesced across lanes; else y = M x (length rows), lane
    // i reads its own row.
    template <bool TR, typename S>
    __device__ __forceinline__ T gmv(const S* M, int rows, int cols, int ld, T x, T* vb) const {
        stage_vec(vb, x);
        return gmv_v<TR>(M, rows, cols, ld, vb);
    }

    // Stage a lane vector in vb (one wave barrier).  Products of vectors
    // staged together then run as gmv_v calls with no barrier between them,
    // so their global loads are issued back to back instead of one product
    // at a time.
    __device__ __forceinline__ void stage_vec(T* vb, T x) const {
        if (lg < NP) vb[lg] = x;
        wg_sync();
    }

    // gmv of a vector already staged in vb (stage_vec)
    template <bool TR, typename S>
    __device__ __forceinline__ T gmv_v(const S* M, int rows, int cols, int ld, const T* vb) const {
        T s = T(0);
        if (TR) {
            if (lg < cols) {
                const S* c = M + lg;
#pragma unroll 4
                for (int i = 0; i < rows; ++i) s = fma_(T(c[(int64_t)i * ld]), vb[i], s);
            }
        } else if (lg < rows) {
            const S* r = M + (int64_t)lg * ld;
            // rows of 16-byte aligned matrices are read 16 bytes at a time
            // (a lane's row is contiguous; lanes read distinct rows)
            constexpr int V = 16 / (int)sizeof(S);
            if ((cols % V) == 0 && (ld % V) == 0 && ((uintptr_t)M & 15) == 0) {
                using S4 = typename std::conditional<sizeof(S) == 4, float4, double2>::type;
                const S4* r4 = reinterpret_cast<const S4*>(r);
#pragma unroll 2
                for (int j = 0; j < cols / V; ++j) {
                    const S4 w = r4[j];
                    if constexpr (sizeof(S) == 4) {
                        s = fma_(T(w.x), vb[4 * j], s);
                        s = fma_(T(w.y), vb[4 * j + 1], s);
                        s = fma_(T(w.z), vb[4 * j + 2], s);
                        s = fma_(T(w.w), vb[4 * j + 3], s);
                    } else {
                        s = fma_(T(w.x), vb[2 * j], s);
                        s = fma_(T(w.y), vb[2 * j + 1], s);
                    }
                }
            } else {
#pragma unroll 4
                for (int j = 0; j < cols; ++j) s = fma_(T(r[j]), vb[j], s);
            }
        }
        return s;
    }

    // gmv_v for the sequential sweeps (one wavefront per instance walking
    // its stages: nothing else on the SIMD hides their load latency): the
    // loads go out in groups (8 column entries, or 5 16-byte row pieces) and
    // the FMAs follow in gmv_v's order, so the result is the same to the bit
    // WIDE: one group for the whole matrix (one wait per product; about 40
    // more registers in flight), for sweeps whose register budget has room
    template <bool TR, bool WIDE = false, typename S>
    __device__ __forceinline__ T gmv_pf(const S* M, int rows, int cols, int ld, const T* vb) const {
        T s = T(0);
        if (TR) {
            constexpr int U = WIDE ? NP : 8;
            // the group loop stays a loop: unrolled, the compiler would
            // hoist every group's loads together (registers past the
            // sweep's budget)
#pragma unroll 1
            for (int i0 = 0; i0 < NP; i0 += U) {
                T c[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    c[u] = (lg < cols && i0 + u < rows) ? T(M[(i0 + u) * ld + lg]) : T(0);
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (i0 + u < rows) s = fma_(c[u], vb[i0 + u], s);
            }
            return lg < cols ? s : T(0);
        }
        constexpr int V = 16 / (int)sizeof(S);
        if ((cols % V) == 0 && (ld % V) == 0 && ((uintptr_t)M & 15) == 0) {
            using S4 = typename std::conditional<sizeof(S) == 4, float4, double2>::type;
            constexpr int NV4 = (NP + V - 1) / V, U = WIDE ? NV4 : 5;
            const S4* r4 = reinterpret_cast<const S4*>(M + (int64_t)lg * ld);
            const int nv = cols / V;
#pragma unroll 1
            for (int j0 = 0; j0 < NV4; j0 += U) {
                S4 w[U];
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (lg < rows && j0 + u < nv) w[u] = r4[j0 + u];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (j0 + u >= nv) break;
                    if constexpr (sizeof(S) == 4) {
                        s = fma_(T(w[u].x), vb[4 * (j0 + u)], s);
                        s = fma_(T(w[u].y), vb[4 * (j0 + u) + 1], s);
                        s = fma_(T(w[u].z), vb[4 * (j0 + u) + 2], s);
                        s = fma_(T(w[u].w), vb[4 * (j0 + u) + 3], s);
                    } else {
                        s = fma_(T(w[u].x), vb[2 * (j0 + u)], s);
                        s = fma_(T(w[u].y), vb[2 * (j0 + u) + 1], s);
                    }
                }
            }
            return lg < rows ? s : T(0);
        }
        return gmv_v<false>(M, rows, cols, ld, vb);
    }

    // --------------------------------------------------------- Cholesky
    // In-register right-looking Cholesky of the n x n SPD matrix held in S
    // (lower triangle used).  On return S holds L (lower, zero above) and
    // lane k's dl holds 1/L_kk (a lane vector).  NV lane vectors in gv are forward-solved
    // with L on the way (gv <- L^{-1} gv).  Returns false if a pivot is not
    // positive (the factorization continues with a unit pivot so values stay
    // finite).  dmin/dmax receive the extreme diagonal entries of L.
    //
    // Step k reads the pivot column straight from the registers of its
    // owner lanes (tx == k % G) with cross-lane reads: the entry of row
    // ty + G a sits in lane (ty, t) as S[a][a0], the entry of row tx + G b in
    // lane (tx, t) as S[b][a0].  No LDS hand-off, no wave barrier per step.
    // NB: the matrix occupies the first NB row/column blocks of the tile
    // (n <= G * NB); the other blocks are left untouched (zero).  cb is
    // unused (kept for the call signature).
    template <int NV, int NB = TS>
    __device__ __forceinline__ bool chol(Tile& S, int n, T* cb, T& dl, T (&gv)[NV > 0 ? NV : 1], T& dmin, T& dmax) const {
        static_assert(NB <= TS, "block limit");
        (void)cb;
        dl = T(1);
        bool ok = true;
        // every pivot root is positive (a failed pivot is replaced by 1), so
        // the running extremes start from the largest finite value and zero
        dmin = sizeof(T) == 4 ? T(3.0e38f) : T(1.0e300);
        dmax = T(0);
#pragma unroll
        for (int a0 = 0; a0 < NB; ++a0) {
            for (int t = 0; t < G; ++t) {
                const int k = G * a0 + t;
                if (k >= n) break;
                const int src_r = ty * G + t;   // lane (ty, t)
                const int src_c = tx * G + t;   // lane (tx, t)
                T cr[NB], cc[NB];
#pragma unroll
                for (int a = 0; a < NB; ++a) cr[a] = __shfl(S[a][a0], src_r, 64);
#pragma unroll
                for (int b2 = a0; b2 < NB; ++b2) cc[b2] = __shfl(S[b2][a0], src_c, 64);
                T d = __shfl(S[a0][a0], t * G + t, 64);
                T gk0[NV > 0 ? NV : 1];
#pragma unroll
                for (int v = 0; v < NV; ++v) gk0[v] = __shfl(gv[v], k, 64);
                const bool good = d > T(0);
                ok = ok && good;
                if (!good) d = T(1);
                T s, inv;
                pivot_root(d, s, inv);
                dmin = s < dmin ? s : dmin;
                dmax = s > dmax ? s : dmax;
                T li[NB], lj[NB];
#pragma unroll
                for (int a = a0; a < NB; ++a) li[a] = cr[a] * inv;
#pragma unroll
                for (int b = a0; b < NB; ++b) lj[b] = cc[b] * inv;
                // In the pivot block only the rows and columns past k take
                // part: their multipliers are zeroed instead of masking the
                // updates (subtracting 0 x leaves an entry as it is).  Blocks
                // past the pivot block lie entirely below and right of k.
                li[a0] = row(a0) > k ? li[a0] : T(0);
                lj[a0] = col(a0) > k ? lj[a0] : T(0);
                // trailing update of the lower triangle: blocks a >= b >= a0
#pragma unroll
                for (int a = a0; a < NB; ++a)
#pragma unroll
                    for (int b = a0; b <= a; ++b) S[a][b] = fma_(-li[a], lj[b], S[a][b]);
                // column k of L; its zeros above the diagonal are the only
                // upper-triangle writes needed: row k right of the diagonal
                // is zeroed by the column writes of the later steps, and the
                // padding past n is zero on entry and stays zero (its
                // multipliers are zero).  Blocks above the pivot block hold
                // rows before k, blocks below it rows after k.
                if (tx == t) {
#pragma unroll
                    for (int a = 0; a < NB; ++a) {
                        if (a < a0) S[a][a0] = T(0);
                        else if (a == a0) S[a][a0] = row(a) == k ? s : li[a];
                        else S[a][a0] = li[a];
                    }
                }
                if (lg == k) dl = inv;
                if (NV > 0) {
                    // element lg of column k (row lg = tx + G ty) is cc[ty]
                    T ck = T(0);
#pragma unroll
                    for (int b = a0; b < NB; ++b)
                        if (ty == b) ck = cc[b];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const T gk = gk0[v] * inv;
                        if (lg == k) gv[v] = gk;
                        else if (lg > k && lg < n) gv[v] = fma_(-ck * inv, gk, gv[v]);
                    }
                }
            }
        }
        wg_sync();
        return ok;
    }

    // ------------------------------------------------ triangular solves
    // X <- L^{-1} X (LOWER=true, forward) or X <- L^{-T} X (LOWER=false,
    // backward with the transpose), L (n x n lower) in LDS slot sL, its
    // reciprocal diagonal as the lane vector dl (lane k: 1/L_kk).  Solves NT register tiles (their first n rows)
    // and NV lane vectors at once.  Step k reads the pivot row from the
    // registers of its owner lanes (ty == k % G; column tx + G b of it sits
    // in lane (t, tx) as X[a0][b]) with cross-lane reads.  rb is unused (kept
    // for the call signature).
    // NB: the solve order n fits the first NB row blocks (n <= G * NB); the
    // rows of the right-hand-side tiles beyond them are left untouched.
    template <bool LOWER, int NT, int NV, int NB = TS>
    __device__ __forceinline__ void trsm(const T* sL, T dl, int n, Tile (&X)[NT > 0 ? NT : 1],
                         T (&vv)[NV > 0 ? NV : 1], T* rb) const {
        static_assert(NB <= TS, "block limit");
        (void)rb;
#pragma unroll
        for (int a0s = 0; a0s < NB; ++a0s) {
            const int a0 = LOWER ? a0s : NB - 1 - a0s;
            for (int ts = 0; ts < G; ++ts) {
                const int t = LOWER ? ts : G - 1 - ts;
                const int k = G * a0 + t;
                if (k >= n) {
                    if (LOWER) break;
                    continue;
                }
                const T dk = lane_at(dl, k);
                const int src = t * G + tx;   // lane (t, tx)
                // rows of blocks past the pivot block are all active (the
                // factor is zero beyond its order n, so no test is needed)
                T lik[NB];
#pragma unroll
                for (int a = 0; a < NB; ++a) {
                    if (LOWER ? a < a0 : a > a0) continue;
                    const int i = row(a);
                    if (a != a0) {
                        lik[a] = LOWER ? sL[i * LD + k] : sL[k * LD + i];
                    } else {
                        const bool act = LOWER ? (i > k && i < n) : (i < k);
                        lik[a] = act ? (LOWER ? sL[i * LD + k] : sL[k * LD + i]) : T(0);
                    }
                }
#pragma unroll
                for (int it = 0; it < NT; ++it) {
                    T rk[TS];
#pragma unroll
                    for (int b = 0; b < TS; ++b) rk[b] = __shfl(X[it][a0][b], src, 64) * dk;
#pragma unroll
                    for (int a = 0; a < NB; ++a) {
                        if (LOWER ? a < a0 : a > a0) continue;
#pragma unroll
                        for (int b = 0; b < TS; ++b)
                            X[it][a][b] = (a == a0 && ty == t) ? rk[b] : fma_(-lik[a], rk[b], X[it][a][b]);
                    }
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T vk = __shfl(vv[v], k, 64) * dk;
                    if (lg == k) vv[v] = vk;
                    else {
                        const bool act = LOWER ? (lg > k && lg < n) : (lg < k);
                        if (act) vv[v] = fma_(-(LOWER ? sL[lg * LD + k] : sL[k * LD + lg]), vk, vv[v]);
                    }
                }
            }
        }
        wg_sync();
    }
};

}  // namespace lqr
