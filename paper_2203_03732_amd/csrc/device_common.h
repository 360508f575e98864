// Device helpers shared by the single-instance and batched phase loops.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prot {

template <class T>
__device__ inline T ld_agent(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline void st_agent(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ inline T add_agent(T *p, T v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// bit e set iff lo <= col0 + e < hi, for e in [0, 8)
__device__ inline uint32_t range_mask(int col0, int lo, int hi)
{
    const int s = lo - col0, t = hi - col0;
    uint32_t m = 0xFFu;
    if (s > 0) m = s >= 8 ? 0u : (m << s) & 0xFFu;
    if (t < 8) m = t <= 0 ? 0u : m & (0xFFu >> (8 - t));
    return m;
}

// bit e set iff k[e] + t[e] == need, i.e. k + 1 == y(a) + y(b) with
// y(a) = -t and need = y(b) - 1.
__device__ inline uint32_t match_mask(uint4 kv, uint4 tv, int need)
{
    const uint32_t kw[4] = {kv.x, kv.y, kv.z, kv.w};
    const uint32_t tw[4] = {tv.x, tv.y, tv.z, tv.w};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int k0 = (int)(int16_t)(kw[i] & 0xFFFFu), k1 = (int)(int16_t)(kw[i] >> 16);
        const int t0 = (int)(tw[i] & 0xFFFFu), t1 = (int)(tw[i] >> 16);
        m |= (uint32_t)(k0 + t0 == need) << (2 * i);
        m |= (uint32_t)(k1 + t1 == need) << (2 * i + 1);
    }
    return m;
}

// Smallest k[e] + t[e] over the elements e whose bit is set in mask (a large
// value if none).
__device__ inline int min_sum_masked(uint4 kv, uint4 tv, uint32_t mask)
{
    const uint32_t kw[4] = {kv.x, kv.y, kv.z, kv.w};
    const uint32_t tw[4] = {tv.x, tv.y, tv.z, tv.w};
    int m = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int s0 = (int)(int16_t)(kw[i] & 0xFFFFu) + (int)(tw[i] & 0xFFFFu);
        const int s1 = (int)(int16_t)(kw[i] >> 16) + (int)(tw[i] >> 16);
        if ((mask >> (2 * i)) & 1u) m = min(m, s0);
        if ((mask >> (2 * i + 1)) & 1u) m = min(m, s1);
    }
    return m;
}

__device__ inline uint32_t lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

struct Hit {
    int j;  // scan position of the hit, -1 if the row is exhausted
    int a;  // its column
};

}  // namespace prot
