// tile_queue.h -- dynamic tiles for the persistent-grid kernels that walk
// the particle arrays tile by tile (the movers, the sort's scatter): the
// live tiles of the segments and the device counters that hand them out.
#pragma once

#include "device_common.h"

namespace picx {

// a block-uniform value moved to scalar registers (the compiler cannot see
// that values read from LDS are the same in every lane)
__device__ __forceinline__ int64_t tq_uniform_i64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Only tiles that hold particles are handed out: segment s has
// ceil(count_s / kTile) of them (none for a subcycled species between its
// pushes), live tile i of the launch is tile i - live0[s] of the segment s
// with live0[s] <= i < live0[s + 1].  Returns their number (all threads; a
// barrier inside; the caller's segment tables in LDS: count[], tile0[],
// live0[], for at most NSEG segments).
template <int NSEG, typename Lds>
__device__ __forceinline__ uint32_t live_tiles_init(Lds &L, const Dev &d)
{
    constexpr int kPerT = NSEG / kBlock;
    static_assert(NSEG % kBlock == 0, "segments per thread");
    const int n = d.n_seg;
    uint32_t v[kPerT];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int sg = threadIdx.x * kPerT + r;
        v[r] = sg < n ? (L.count[sg] + (uint32_t)kTile - 1u) / (uint32_t)kTile : 0u;
        sum += v[r];
    }
    __shared__ uint32_t s_w[kWaves];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int w = 0; w < wave; ++w) run += s_w[w];
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int sg = threadIdx.x * kPerT + r;
        if (sg <= n) L.live0[sg] = run;
        run += v[r];
    }
    if (threadIdx.x == kBlock - 1) L.live0[n] = run;  // (n = NSEG: no thread above wrote it)
    __syncthreads();
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)L.live0[n]);
}

// the tile of live tile i; hint: the segment of the previous one (they only
// increase), so a few steps forward usually find it, else a binary search
template <int NSEG, typename Lds>
__device__ __forceinline__ int64_t live_tile(const Lds &L, const Dev &d, uint32_t i, int &hint)
{
    if (d.n_seg > NSEG) return (int64_t)i;  // no tables: every tile, empty ones included
    int sg = hint, steps = 0;
    while (sg + 1 < d.n_seg && L.live0[sg + 1] <= i && steps < 8) {
        ++sg;
        ++steps;
    }
    if (sg + 1 < d.n_seg && L.live0[sg + 1] <= i) {
        int lo = sg, hi = d.n_seg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.live0[mid] <= i) lo = mid; else hi = mid - 1;
        }
        sg = lo;
    }
    sg = __builtin_amdgcn_readfirstlane(sg);
    hint = sg;
    return tq_uniform_i64(L.tile0[sg] + (int64_t)(i - L.live0[sg]));
}

// The movers and the sort's scatter take their tiles dynamically, so that a
// block slowed by where its tiles lie in memory does not hold up the
// launch.  Tiles are counted among the live ones (live_tiles_init).  Block b
// starts on live tile b; the tiles past the grid are handed out by
// K = min(kUnitCtrs, blocks) counters, interleaved (counter k: tiles
// blocks + k, blocks + k + K, ...), so that the taken tiles still form one
// front sweeping the arrays; block b takes from counter b % K.  Wave 0
// issues the grab for the block's next tile once the loads of the tile in
// hand are issued (tile_grab; on one in-order memory counter, a grab issued
// before them would hold them up), else at the end of the tile, and hands
// the result to the other waves through LDS at a block barrier.  A block
// whose grab finds the counter exhausted issues no more and adds itself to
// the counter's done count; the last block of the counter's group sets both
// back to zero for the next launch (no grab of this launch can follow: every
// block of the group has made its last).
struct TileQueue {
    unsigned int *ctr;   // [0]: grabs, [1]: blocks done
    uint32_t n_mine;     // tiles of this counter
    uint32_t n_blocks;   // blocks taking from this counter
    uint32_t k, K, first;
    uint32_t pending;    // the last grab (lane 0 of wave 0)
    bool grabbed;        // a grab was issued since the last tile was taken
};

__device__ __forceinline__ void tile_queue_init(TileQueue &Q, const Dev &d, uint32_t nt)
{
    const uint32_t nb = gridDim.x;
    Q.K = nb < (uint32_t)kUnitCtrs ? nb : (uint32_t)kUnitCtrs;
    Q.k = blockIdx.x % Q.K;
    Q.first = nb;
    Q.ctr = d.glob->unit_ctr + Q.k * kUnitCtrStride;
    const uint32_t rest = nt > nb ? nt - nb : 0u;
    Q.n_mine = rest > Q.k ? (rest - Q.k + Q.K - 1) / Q.K : 0u;
    Q.n_blocks = (nb - Q.k + Q.K - 1) / Q.K;
    Q.pending = 0u;
    Q.grabbed = false;
}

// The result is first read by tile_next, so that no wait for it holds up
// the work on the loads issued ahead of it.  (An increment that wraps at
// 2^32 - 1, never reached: the compiler aggregates a uniform atomicAdd over
// the wave and reads its result at once, which would wait for every load in
// flight.)
__device__ __forceinline__ void tile_grab(TileQueue &Q)
{
    if (lane_id() == 0) Q.pending = atomicInc(Q.ctr, 0xFFFFFFFFu);
    Q.grabbed = true;
}

// the block's next live tile (an index for live_tile), -1 when its counter
// is exhausted (wave 0)
__device__ __forceinline__ int64_t tile_next(TileQueue &Q)
{
    if (!Q.grabbed) tile_grab(Q);
    Q.grabbed = false;
    const uint32_t i = (uint32_t)__builtin_amdgcn_readfirstlane((int)Q.pending);
    if (i >= Q.n_mine) {
        if (lane_id() == 0 && atomicAdd(Q.ctr + 1, 1u) == Q.n_blocks - 1u) {
            atomicExch(Q.ctr, 0u);
            atomicExch(Q.ctr + 1, 0u);
        }
        return -1;
    }
    return (int64_t)Q.first + Q.k + (int64_t)i * Q.K;
}

}  // namespace picx
