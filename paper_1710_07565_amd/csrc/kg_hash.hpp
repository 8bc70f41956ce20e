// kg_hash.hpp -- an order-independent 64-bit checksum of an edge list, for a
// consumer that checks what it received on the device instead of copying
// the list to the host:
//   h = sum over i of mix(i * 0x9E3779B97F4A7C15 + (u_i << 32 | v_i))  mod 2^64,
// mix = the finaliser of SplitMix64 (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014).  Every term depends on the
// edge and its position, so a changed, missing or moved edge changes h; the
// sum makes the result independent of how the work is split.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kg {

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t edge_term(uint64_t i, uint32_t u, uint32_t v)
{
    return mix64(i * 0x9E3779B97F4A7C15ull + (((uint64_t)u << 32) | v));
}

// The accumulator is cleared by a kernel (not a memset), so the pair can be
// recorded into a graph.
__global__ void hash_clear_kernel(uint64_t *out) { if (threadIdx.x == 0 && blockIdx.x == 0) *out = 0; }

// Grid-stride over pairs of edges (one 16-byte load per lane), a wave sum,
// one 64-bit atomic add per wave.  A list starting at an odd 8-byte address
// takes its first edge on its own, so the pairs are 16-byte aligned.
__global__ __launch_bounds__(256) void hash_kernel(const uint32_t *edges, uint64_t n, uint64_t *out)
{
    const uint64_t lead = (((uintptr_t)edges & 15) != 0 && n > 0) ? 1 : 0;
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint64_t npair = (n - lead) >> 1;
    const uint4 *e4 = reinterpret_cast<const uint4 *>(edges + 2 * lead);
    uint64_t acc = 0;
    for (uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x; j < npair; j += stride) {
        const uint4 q = e4[j];
        const uint64_t i = lead + 2 * j;
        acc += edge_term(i, q.x, q.y) + edge_term(i + 1, q.z, q.w);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (lead) acc += edge_term(0, edges[0], edges[1]);
        if (((n - lead) & 1) != 0) {
            const uint64_t i = n - 1;
            acc += edge_term(i, edges[2 * i], edges[2 * i + 1]);
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd((unsigned long long *)out, (unsigned long long)acc);
}

}  // namespace kg
