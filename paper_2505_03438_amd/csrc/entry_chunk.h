// Eight pending 16-bit list entries in four words, written to memory as one
// 16-byte chunk: after eight pushes entry 2k sits in the low half of word k
// and entry 2k + 1 in the high half.  Used by the list builds that store
// their entries in chunks of eight (the batched Verlet lists and the Verlet
// list cells).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mdlj {

struct EntryChunk {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    __device__ __forceinline__ void push(uint32_t e)
    {
        w[0] = (w[0] >> 16) | (w[1] << 16);
        w[1] = (w[1] >> 16) | (w[2] << 16);
        w[2] = (w[2] >> 16) | (w[3] << 16);
        w[3] = (w[3] >> 16) | (e << 16);
    }
    __device__ __forceinline__ uint4 word() const { return make_uint4(w[0], w[1], w[2], w[3]); }
};

// Entry u (0..7) of a chunk.
__device__ __forceinline__ uint32_t chunk_entry(const uint4 &c, int u)
{
    const uint32_t w = u < 2 ? c.x : (u < 4 ? c.y : (u < 6 ? c.z : c.w));
    return (w >> (16 * (u & 1))) & 0xffffu;
}

}  // namespace mdlj
