// pack.hpp -- gather / scatter kernels of ragged batches (problems of one
// shape packed into a contiguous batch and back).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lqr {

// Packing of ragged batches: up to kPackTable problems per launch, their
// device pointers passed as kernel arguments.  GATHER: packed[j][w] =
// one_j[w]; else one_j[w] = packed[j][w], over `words` 32-bit words per
// problem (every array holds 4- or 8-byte elements).
constexpr int kPackTable = 48;
struct PackTable {
    void* p[kPackTable];
    int idx[kPackTable];
    int count;
};

template <bool GATHER>
__global__ void k_pack(PackTable t, uint32_t* packed, int64_t words) {
    const int j = blockIdx.y;
    if (j >= t.count) return;
    uint32_t* one = static_cast<uint32_t*>(t.p[j]);
    uint32_t* pk = packed + (int64_t)j * words;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
        if (GATHER) pk[w] = one[w];
        else one[w] = pk[w];
    }
}

// status / residual of packed problem j back to descriptor position idx[j]
template <typename D>
__global__ void k_unpack_status(PackTable t, const int32_t* st, const D* rel, int32_t* status_out, D* rel_out) {
    const int j = threadIdx.x;
    if (j >= t.count) return;
    status_out[t.idx[j]] = st[j];
    if (rel_out) rel_out[t.idx[j]] = rel[j];
}

}  // namespace lqr
