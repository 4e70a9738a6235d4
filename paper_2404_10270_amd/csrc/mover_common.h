// mover_common.h -- pieces of the mover shared by libpic (push.hip) and the
// layout study (study/layout.hip): streaming loads and stores, wave
// reductions, and the deposit through a per-wave LDS window of nodes.
#pragma once

#include "device_common.h"

namespace picx {

// Particle arrays are streamed once per step (the state is far larger than
// the caches): nontemporal loads and stores keep them from displacing the
// grid, the deposit window flushes and the candidate regions in L2.
template <typename T>
__device__ __forceinline__ T stream_ld(const T *p)
{
    return __builtin_nontemporal_load(p);
}

template <typename T>
__device__ __forceinline__ void stream_st(T *p, T v)
{
    __builtin_nontemporal_store(v, p);
}

// Orders this wave's LDS operations before and after the call (a wave's LDS
// operations complete in issue order; the fences keep the compiler from
// moving them across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kWaveWin = 64;      // LDS deposit window of one wave, nodes

// Deposit the NP chunks of this wave through its own LDS window
// wdep[kWaveWin] (zero between calls), with no block barrier: runs of equal
// cells are summed across lanes, their two node weights added into the
// window, and the window flushed with one 64-bit global atomic per touched
// node.  A run whose nodes fall outside the window adds to S directly.
// In two halves, so that a mover can issue its next tile's loads between
// them: deposit_accumulate fills the window (span = 0: nothing to flush),
// deposit_flush adds it to S and clears it.  The window's bounds come from
// DPP lane moves (no LDS round trip).
template <int NP>
__device__ __forceinline__ void deposit_accumulate(unsigned long long *wdep, unsigned long long *__restrict__ S,
                                                   const int (&key)[NP], const unsigned long long (&w1)[NP],
                                                   int &lo, int &span)
{
    int kmn = 0x7fffffff, kmx = -1;
#pragma unroll
    for (int k = 0; k < NP; ++k)
        if (key[k] >= 0) {
            kmn = min(kmn, key[k]);
            kmx = max(kmx, key[k]);
        }
    lo = wave_reduce_dpp<false>(kmn);
    const int hi = wave_reduce_dpp<true>(kmx);
    span = 0;
    if (hi < 0) return;  // no live particle in the wave's chunks
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        // pack (count, sum W1): W1 <= 2^32 and at most 64 lanes -> sum < 2^39
        const unsigned long long v = (key[k] >= 0) ? ((1ull << 40) + w1[k]) : 0ull;
        bool tail;
        const unsigned long long t = run_sum(key[k], v, tail);
        if (tail && key[k] >= 0) {
            const unsigned long long n = t >> 40;
            const unsigned long long b = t & ((1ull << 40) - 1ull);
            const unsigned long long a = (n << PIC_FRAC_BITS) - b;
            const int rel = key[k] - lo;
            if (rel + 1 < kWaveWin) {
                atomicAdd(&wdep[rel], a);
                atomicAdd(&wdep[rel + 1], b);
            } else {
                atomicAdd(S + key[k], a);
                atomicAdd(S + key[k] + 1, b);
            }
        }
    }
    span = min(hi - lo + 2, kWaveWin);
}

__device__ __forceinline__ void deposit_flush(unsigned long long *wdep, unsigned long long *__restrict__ S, int lo,
                                              int span)
{
    static_assert(kWaveWin == 64, "one window node per lane");
    wave_lds_sync();
    const int i = lane_id();
    if (i < span) {
        const unsigned long long v = wdep[i];
        if (v) {
            atomicAdd(S + lo + i, v);
            wdep[i] = 0ull;
        }
    }
    wave_lds_sync();
}

template <int NP>
__device__ __forceinline__ void deposit_wave(unsigned long long *wdep, unsigned long long *__restrict__ S,
                                             const int (&key)[NP], const unsigned long long (&w1)[NP])
{
    int lo, span;
    deposit_accumulate<NP>(wdep, S, key, w1, lo, span);
    if (span > 0) deposit_flush(wdep, S, lo, span);
}

}  // namespace picx
