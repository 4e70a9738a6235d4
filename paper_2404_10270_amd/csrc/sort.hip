// sort.hip -- "natural sorting" (paper Sec. 2: particles stored grouped by
// the cell they occupy) as a counting sort by cell into the other buffer set,
// dropping absorbed particles (gfx950).
//
//   hist     one bin per (species, node) counts the live particles of each
//            cell; every wave first counts its chunks of a tile into its own
//            LDS window of bins (wave-level run sums, then LDS atomics, no
//            block barrier) and adds the window to the global bins with one
//            atomic per touched bin
//   scan     single-pass exclusive scan of all bins (decoupled look-back);
//            writes the scatter cursors and the per-segment cell offsets
//   scatter  every tile ranks its particles per bin in LDS, reserves each
//            bin's share with one global atomic per touched bin, and copies
//            the particles to the other set
//   finish   one block switches the current set and sets the counts
// The scatter also records the largest |vx| of a kinetic neutral species:
// atoms keep their velocity until the next sort, so it bounds how far any
// of them can move from the cell the offsets list it in.
// Segment starts come from the live counts, so absorbed particles need no bin.
#include <type_traits>

#include "device_common.h"
#include "tile_queue.h"

namespace picx {

constexpr int kSortWin = 1024;  // LDS window of bins per tile (scatter)
constexpr int kHistWaveWin = 64;  // LDS window of bins per wave (histogram)

// orders this wave's LDS operations before and after the call (a wave's LDS
// operations complete in issue order; the fences keep the compiler from
// moving them across)
__device__ __forceinline__ void hist_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
constexpr int kSegLdsS = 1024;

struct SortLds {
    uint32_t cnt[kSortWin];
    uint32_t base[kSortWin];
    int64_t tile0[kSegLdsS + 1];
    int64_t sbase[kSegLdsS];
    uint32_t count[kSegLdsS];
    uint32_t live0[kSegLdsS + 1];  // the scatter: live tiles of the segments before each
    int red[2][kWaves];
};

__device__ __forceinline__ void sort_lds_init(SortLds &L, const Dev &d)
{
    for (int i = threadIdx.x; i < kSortWin; i += kBlock) L.cnt[i] = 0u;
    if (d.n_seg <= kSegLdsS) {
        for (int s = threadIdx.x; s <= d.n_seg; s += kBlock) {
            L.tile0[s] = d.seg_tile0[s];
            if (s < d.n_seg) {
                L.sbase[s] = d.seg_base[s];
                L.count[s] = d.segd[s].count;
            }
        }
    }
    __syncthreads();
}

// hint: the segment of the block's previous tile (tiles only increase)
__device__ __forceinline__ int sort_tile_seg(const SortLds &L, const Dev &d, int64_t t,
                                             int64_t &tile0, int64_t &base, int64_t &count,
                                             int &hint)
{
    int seg;
    if (d.n_seg <= kSegLdsS) {
        int s = hint, steps = 0;
        while (s + 1 < d.n_seg && L.tile0[s + 1] <= t && steps < 8) {
            ++s;
            ++steps;
        }
        if (s + 1 < d.n_seg && L.tile0[s + 1] <= t) {
            int lo = s, hi = d.n_seg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.tile0[mid] <= t) lo = mid; else hi = mid - 1;
            }
            s = lo;
        }
        seg = __builtin_amdgcn_readfirstlane(s);
        hint = seg;
        tile0 = L.tile0[seg];
        base = L.sbase[seg];
        count = L.count[seg];
    } else {
        seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        tile0 = d.seg_tile0[seg];
        base = d.seg_base[seg];
        count = d.segd[seg].count;
    }
    return seg;
}

// Runs of equal keys in lane order (a run: a maximal group of consecutive
// lanes with one key).  Returns the lane's 1-based position in its run;
// is_tail marks the run's last lane, whose position is the run's length
// (the count of particles in one cell, as every lane of a run of live keys
// counts one).
__device__ __forceinline__ uint32_t run_position(int key, bool &is_tail)
{
    const int lane = lane_id();
    const int up = __shfl_up(key, 1, 64);
    const int dn = __shfl_down(key, 1, 64);
    const bool head = (lane == 0) || (up != key);
    is_tail = (lane == 63) || (dn != key);
    const unsigned long long heads = ballot(head);
    const unsigned long long mask = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
    return (uint32_t)(lane - (63 - __clzll(mask)) + 1);
}

// block window [lo, hi] over the keys of this tile (barrier inside)
__device__ __forceinline__ void tile_window(SortLds &L, const int (&key)[kPer], int &lo, int &hi)
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    int kmn = 0x7fffffff, kmx = -1;
#pragma unroll
    for (int k = 0; k < kPer; ++k)
        if (key[k] >= 0) {
            kmn = min(kmn, key[k]);
            kmx = max(kmx, key[k]);
        }
    kmn = wave_reduce_dpp<false>(kmn);
    kmx = wave_reduce_dpp<true>(kmx);
    if (lane == 0) {
        L.red[0][wave] = kmn;
        L.red[1][wave] = kmx;
    }
    __syncthreads();
    lo = L.red[0][0];
    hi = L.red[1][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
        lo = min(lo, L.red[0][w]);
        hi = max(hi, L.red[1][w]);
    }
}

// the block's first tile holding particles at or after tile t (its stride:
// the grid), -1 when none; its segment's values in seg, base, count, t0
__device__ __forceinline__ int64_t hist_next_tile(const SortLds &L, const Dev &d, int64_t t, int &seg,
                                                  int64_t &base, int64_t &count, int64_t &t0, int &hint)
{
    for (; t < d.n_tiles; t += gridDim.x) {
        int64_t tile0;
        seg = sort_tile_seg(L, d, t, tile0, base, count, hint);
        t0 = (t - tile0) * (int64_t)kTile;
        if (t0 < count) return t;
    }
    return -1;
}

// The raw keys of a wave's kPer chunks of a tile (in-segment slots
// t0 + 64 (wave kPer + k) + lane): the cell (FP32 form) or the position
// (FP64 form).  Slots past the segment's count load the tile's first slot
// instead (their keys are -1), so that every tile issues the same loads.
template <bool F64>
using RawKey = typename std::conditional<F64, double, int32_t>::type;

template <bool F64>
__device__ __forceinline__ void load_raw_keys(const Dev &d, int cur, int64_t base, int64_t t0, int64_t count,
                                              RawKey<F64> (&raw)[kPer])
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const RawKey<F64> *src = F64 ? (const RawKey<F64> *)d.x[cur] : (const RawKey<F64> *)d.cell[cur];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
        raw[k] = __builtin_nontemporal_load(&src[base + (i < count ? i : t0)]);
    }
}

template <bool F64>
__device__ __forceinline__ void raw_to_keys(const RawKey<F64> (&raw)[kPer], int64_t t0, int64_t count,
                                            int (&key)[kPer])
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const bool in = t0 + (int64_t)(wave * kPer + k) * 64 + lane < count;
        if (F64) key[k] = in && raw[k] >= 0.0 ? (int)floor((double)raw[k]) : -1;
        else key[k] = in ? (int)raw[k] : -1;
    }
}

// Each wave requests its chunks of the block's next tile (and that tile's
// segment values) before it adds the counts of the tile in hand to the
// global bins: the loads and the atomics are then in flight together,
// rather than each tile's loads waiting behind the previous tile's atomics
// on the in-order memory counter.  Every pass issues the same loads (the
// last one repeats its own tile's), so the wait for the tile in hand leaves
// the next tile's loads in flight.
template <bool F64>
__global__ __launch_bounds__(kBlock) void sort_hist_kernel(Dev d)
{
    __shared__ SortLds L;
    __shared__ uint32_t wcnt[kWaves][kHistWaveWin];  // each wave's window of bins
    for (int i = threadIdx.x; i < kWaves * kHistWaveWin; i += kBlock) (&wcnt[0][0])[i] = 0u;
    sort_lds_init(L, d);
    const int cur = d.glob->cur_set;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t *W = wcnt[wave];
    int hint = 0;  // segment of the previous tile
    int seg = 0;
    int64_t base = 0, count = 0, t0 = 0;
    int64_t t = hist_next_tile(L, d, blockIdx.x, seg, base, count, t0, hint);
    if (t < 0) return;
    // the segment's bins: species and first node, read beside its keys
    int sp = d.segc[seg].sp;
    int64_t gnode = d.segc[seg].gnode;
    RawKey<F64> raw[kPer];
    load_raw_keys<F64>(d, cur, base, t0, count, raw);
    while (t >= 0) {
        int nseg = seg;
        int64_t nbase = base, ncount = count, nt0 = t0;
        const int64_t tn = hist_next_tile(L, d, t + gridDim.x, nseg, nbase, ncount, nt0, hint);
        if (tn < 0) {  // (no next tile: the loads repeat this one's, unused)
            nseg = seg;
            nbase = base;
            ncount = count;
            nt0 = t0;
        }
        const int nsp = d.segc[nseg].sp;
        const int64_t ngnode = d.segc[nseg].gnode;
        RawKey<F64> nraw[kPer];
        load_raw_keys<F64>(d, cur, nbase, nt0, ncount, nraw);
        int key[kPer];
        raw_to_keys<F64>(raw, t0, count, key);
        uint32_t *__restrict__ H = d.hist + (int64_t)sp * d.G + gnode;
        // this wave's bins: run sums of equal keys into its own LDS window (no
        // block barrier), then one global atomic per touched bin
        int kmn = 0x7fffffff, kmx = -1;
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (key[k] >= 0) {
                kmn = min(kmn, key[k]);
                kmx = max(kmx, key[k]);
            }
        const int lo = wave_reduce_dpp<false>(kmn);
        const int hi = wave_reduce_dpp<true>(kmx);
        if (hi >= 0) {  // (else no live particle in the wave's chunks)
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                bool tail;
                const uint32_t n = run_position(key[k], tail);
                if (tail && key[k] >= 0) {
                    const int rel = key[k] - lo;
                    if (rel >= 0 && rel < kHistWaveWin) atomicAdd(&W[rel], n);
                    else atomicAdd(H + key[k], n);
                }
            }
            hist_wave_sync();
            static_assert(kHistWaveWin == 64, "one window bin per lane");
            const int span = min(hi - lo + 1, kHistWaveWin);
            if (lane < span) {
                const uint32_t v = W[lane];
                if (v) {
                    atomicAdd(H + lo + lane, v);
                    W[lane] = 0u;
                }
            }
            hist_wave_sync();
        }
        t = tn;
        seg = nseg;
        base = nbase;
        count = ncount;
        t0 = nt0;
        sp = nsp;
        gnode = ngnode;
#pragma unroll
        for (int k = 0; k < kPer; ++k) raw[k] = nraw[k];
    }
}

__device__ __forceinline__ void st_rel(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(kBlock) void sort_scan_kernel(Dev d)
{
    __shared__ uint32_t s_t;
    __shared__ unsigned long long s_g;
    if (threadIdx.x == 0) {
        s_g = __hip_atomic_load(&d.glob->scan_gen[kScanSort], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
        s_t = atomicAdd(&d.glob->scan_ticket[kScanSort], 1u);
    }
    __syncthreads();
    const int64_t vt = s_t;
    const unsigned long long gen = s_g;
    const int64_t nbins = (int64_t)d.nsp * d.G;
    const int64_t b0 = vt * kSortTile + (int64_t)threadIdx.x * kSortR;
    uint32_t h[kSortR];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kSortR; ++r) {
        const int64_t b = b0 + r;
        h[r] = (b < nbins) ? d.hist[b] : 0u;
        if (b < nbins) d.hist[b] = 0u;  // ready for the next sort
        sum += h[r];
    }
    // block exclusive scan of the thread sums
    __shared__ uint32_t s_w[kWaves];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t inc = sum;
#pragma unroll
    for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t o = __shfl_up(inc, dd, 64);
        if (lane >= dd) inc += o;
    }
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
    for (int w = 0; w < kWaves; ++w) {
        if (w < wave) wpre += s_w[w];
        total += s_w[w];
    }
    const uint32_t excl = wpre + inc - sum;
    // look-back: flag word = gen << 34 | state << 32 | value
    __shared__ uint32_t s_in;
    if (threadIdx.x == 0) {
        unsigned long long *st = d.sort_status;
        uint32_t in = 0;
        if (vt == 0) {
            st_rel(&st[0], (gen << 34) | (2ull << 32) | total);
        } else {
            st_rel(&st[vt], (gen << 34) | (1ull << 32) | total);
            for (int64_t p = vt - 1;; --p) {
                unsigned long long f;
                do {
                    f = __hip_atomic_load(&st[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } while ((f >> 34) != gen);
                in += (uint32_t)f;
                if (((f >> 32) & 3ull) == 2ull) break;
            }
            st_rel(&st[vt], (gen << 34) | (2ull << 32) | (uint32_t)(in + total));
        }
        s_in = in;
    }
    __syncthreads();
    uint32_t run = s_in + excl;
    // rebasing per segment: bin b belongs to species b / G and the instance owning node b % G
#pragma unroll
    for (int r = 0; r < kSortR; ++r) {
        const int64_t b = b0 + r;
        if (b < nbins) {
            d.cursor[b] = run;
            const int sp = (int)(b / d.G);
            const int64_t node = b - (int64_t)sp * d.G;
            const int inst = seg_of_tile(d.node_base, d.n_inst, node);
            const int seg = inst * d.nsp + sp;
            d.offsets[b] = run - (uint32_t)d.seg_start[seg];
        }
        run += h[r];
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&d.glob->scan_finish[kScanSort], 1u);
        if ((int64_t)prev == d.n_sort_tiles - 1) {
            d.glob->scan_ticket[kScanSort] = 0;
            d.glob->scan_finish[kScanSort] = 0;
            d.glob->scan_gen[kScanSort] = d.glob->scan_gen[kScanSort] + 1ull;
            __threadfence();
        }
    }
}

// The fields of a wave's kPer chunks of a tile (in-segment slots
// t0 + 64 (wave kPer + k) + lane): the cell (FP32 form) or the position
// (FP64 form) first, the key being made from it, then the rest.  Slots past
// the segment's count load the tile's first slot instead (never stored), so
// that every tile issues the same loads and the waits for them are counted
// exactly.  The source arrays are streamed once per sort: nontemporal loads
// keep them from displacing the bins, cursors and the scattered
// destinations in L2 (the stores stay cached: a tile's particles go to many
// bins, and L2 merges their partial lines).
template <bool F64>
struct TileFields {
    using V = typename std::conditional<F64, double, float>::type;
    V x[kPer], vx[kPer], vy[kPer], vz[kPer];
    int32_t c[kPer];
    uint32_t lo[kPer], hi[kPer];
};

template <bool F64>
__device__ __forceinline__ void load_fields(const Dev &d, int cur, int64_t base, int64_t t0, int64_t count,
                                            TileFields<F64> &F, bool (&in)[kPer])
{
    using V = typename TileFields<F64>::V;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const V *X = (const V *)d.x[cur], *VX = (const V *)d.vx[cur], *VY = (const V *)d.vy[cur],
            *VZ = (const V *)d.vz[cur];
    int64_t g[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
        in[k] = i < count;
        g[k] = base + (in[k] ? i : t0);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (F64) F.x[k] = __builtin_nontemporal_load(&X[g[k]]);
        else F.c[k] = __builtin_nontemporal_load(&d.cell[cur][g[k]]);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (!F64) F.x[k] = __builtin_nontemporal_load(&X[g[k]]);
        F.vx[k] = __builtin_nontemporal_load(&VX[g[k]]);
        F.vy[k] = __builtin_nontemporal_load(&VY[g[k]]);
        F.vz[k] = __builtin_nontemporal_load(&VZ[g[k]]);
        F.lo[k] = __builtin_nontemporal_load(&d.id_lo[cur][g[k]]);
        F.hi[k] = __builtin_nontemporal_load(&d.id_hi[cur][g[k]]);
    }
}

// the stores of the particles with a destination (to[k] >= 0) to the other set
template <bool F64>
__device__ __forceinline__ void store_fields(const Dev &d, int nxt, const TileFields<F64> &F,
                                             const int64_t (&to)[kPer])
{
    using V = typename TileFields<F64>::V;
    V *Xn = (V *)d.x[nxt], *VXn = (V *)d.vx[nxt], *VYn = (V *)d.vy[nxt], *VZn = (V *)d.vz[nxt];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (to[k] < 0) continue;
        const int64_t t = to[k];
        Xn[t] = F.x[k];
        VXn[t] = F.vx[k];
        VYn[t] = F.vy[k];
        VZn[t] = F.vz[k];
        if (!F64) d.cell[nxt][t] = F.c[k];
        d.id_lo[nxt][t] = F.lo[k];
        d.id_hi[nxt][t] = F.hi[k];
    }
}

// rank of each of the wave's particles among the tile's particles of its
// cell: in-window bins count in LDS; a bin outside the tile's window
// (OUT: some key of the wave is outside) is reserved directly with a global
// atomic.  Two forms, so that the common one holds no global atomic whose
// result the compiler would wait for together with the fields in flight.
template <bool OUT>
__device__ __forceinline__ void tile_ranks(SortLds &L, uint32_t *__restrict__ CUR, const int (&key)[kPer],
                                           int lo, const bool (&outside)[kPer], uint32_t (&rank)[kPer])
{
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        bool tail;
        const uint32_t inc = run_position(key[k], tail);
        const unsigned long long tails = ballot(tail);
        uint32_t rb = 0;
        if (tail && key[k] >= 0) {
            if (!OUT || !outside[k]) rb = atomicAdd(&L.cnt[key[k] - lo], (uint32_t)inc);
            else rb = atomicAdd(CUR + key[k], (uint32_t)inc);
        }
        const unsigned long long above = tails & ~((1ull << lane) - 1ull);
        const int tl = __ffsll((long long)above) - 1;
        rb = __shfl(rb, tl, 64);
        rank[k] = rb + (uint32_t)inc - 1u;
    }
}

// Each tile's fields are all loaded first, and stay in registers while the
// tile ranks its particles and reserves its bins: the loads are in flight
// during the ranks, and the wait for the reservations' returns covers them
// too, rather than the loads starting only once the destinations are known.
// (held to four waves per SIMD: the grid is one residency of 4 blocks per CU)
template <bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void sort_scatter_kernel(Dev d)
{
    __shared__ SortLds L;
    sort_lds_init(L, d);
    const int cur = d.glob->cur_set;
    const int nxt = cur ^ 1;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    int hint = 0;  // segment of the previous tile
    // tiles taken dynamically (tile_queue.h); the next one is handed on at
    // the barrier after the reservations
    const uint32_t n_live = d.n_seg <= kSegLdsS ? live_tiles_init<kSegLdsS>(L, d) : (uint32_t)d.n_tiles;
    TileQueue Q;
    tile_queue_init(Q, d, n_live);
    int lhint = 0;  // segment of the previous live tile
    __shared__ int64_t s_next[2];  // the block's next tile, by parity of its tiles
    int par = 0;
    const bool w0 = __builtin_amdgcn_readfirstlane(wave) == 0;
    auto hand_on = [&]() {
        if (w0) {
            const int64_t i = tile_next(Q);
            const int64_t n = i >= 0 ? live_tile<kSegLdsS>(L, d, (uint32_t)i, lhint) : -1;
            if (lane == 0) s_next[par] = n;
        }
    };
    int64_t t = blockIdx.x < n_live ? live_tile<kSegLdsS>(L, d, blockIdx.x, lhint) : -1;
    if (t >= 0) do {
        int64_t tile0, base, count;
        const int seg = sort_tile_seg(L, d, t, tile0, base, count, hint);
        const int64_t t0 = (t - tile0) * (int64_t)kTile;
        if (t0 >= count) {  // (only without the LDS tables: every tile is handed out)
            hand_on();
            __syncthreads();
            t = tq_uniform_i64(s_next[par]);
            par ^= 1;
            continue;
        }
        // the segment's values read before the fields (in the order of the
        // memory counter, no wait for them then waits for the fields)
        const SegConst &sc = d.segc[seg];
        const uint32_t start = (uint32_t)d.seg_start[seg];
        uint32_t *__restrict__ CUR = d.cursor + sc.sp * d.G + sc.gnode;
        const uint32_t cap = sc.cap;
        const int64_t sbase = sc.base;
        const bool neutral = sc.kind == PIC_KIND_NEUTRAL;
        TileFields<F64> F;
        bool in[kPer];
        load_fields<F64>(d, cur, base, t0, count, F, in);
        if (w0) tile_grab(Q);  // the next tile, behind this one's loads
        int key[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (F64) key[k] = in[k] && F.x[k] >= 0.0 ? (int)floor((double)F.x[k]) : -1;
            else key[k] = in[k] ? F.c[k] : -1;
        }
        int lo, hi;
        tile_window(L, key, lo, hi);
        // rank of every particle among the tile's particles of its cell
        uint32_t rank[kPer];
        bool outside[kPer], any_out = false;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            outside[k] = key[k] >= 0 && (key[k] < lo || key[k] - lo >= kSortWin);
            any_out = any_out || outside[k];
        }
        if (ballot(any_out)) tile_ranks<true>(L, CUR, key, lo, outside, rank);
        else tile_ranks<false>(L, CUR, key, lo, outside, rank);
        __syncthreads();
        // one global reservation per touched bin
        if (hi >= 0) {
            const int span = min(hi - lo + 1, kSortWin);
            for (int i = threadIdx.x; i < span; i += kBlock) {
                const uint32_t v = L.cnt[i];
                if (v) {
                    L.base[i] = atomicAdd(CUR + lo + i, v);
                    L.cnt[i] = 0u;
                }
            }
        }
        hand_on();
        __syncthreads();
        const int64_t t_next = tq_uniform_i64(s_next[par]);
        par ^= 1;
        int64_t to[kPer];
        bool overflow = false;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            to[k] = -1;
            if (key[k] < 0) continue;
            const uint32_t pos = outside[k] ? rank[k] : L.base[key[k] - lo] + rank[k];
            const uint32_t rel = pos - start;
            if (rel >= cap) {  // cannot happen with a consistent histogram
                overflow = true;
                continue;
            }
            to[k] = sbase + (int64_t)rel;
        }
        if (overflow) atomicOr(&d.instd[sc.inst].status, PIC_ST_INTERNAL);
        store_fields<F64>(d, nxt, F, to);
        if (neutral) {
            unsigned long long vb = 0ull;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                if (key[k] < 0) continue;
                const unsigned long long b =
                    (unsigned long long)__double_as_longlong(fabs((double)F.vx[k]));
                vb = b > vb ? b : vb;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const uint32_t lo = __shfl_xor((uint32_t)vb, o, 64);
                const uint32_t hi = __shfl_xor((uint32_t)(vb >> 32), o, 64);
                const unsigned long long w = ((unsigned long long)hi << 32) | lo;
                vb = w > vb ? w : vb;
            }
            // same-address atomics serialise: only a wave that raises the
            // maximum it can see issues one
            unsigned long long *vm = &d.segd[seg].vmax_bits;
            if (lane == 0 && vb > __hip_atomic_load(vm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(vm, vb);
        }
        // the next tile's window barrier orders the reuse of L.base
        t = t_next;
    } while (t >= 0);
    else if (w0) (void)tile_next(Q);  // (no tile for this block: its counter still counts it done)
}

// after the scatter (one block): switch sets and set the counts to the live particles
__global__ void sort_finish_kernel(Dev d)
{
    for (int s = threadIdx.x; s < d.n_seg; s += blockDim.x) {
        const SegConst &sc = d.segc[s];
        // offsets[node nc] of the segment = particles in its cell bins
        const uint32_t n_live = d.offsets[sc.sp * d.G + sc.gnode + sc.nc];
        if (n_live != d.segd[s].live) atomicOr(&d.instd[sc.inst].status, PIC_ST_INTERNAL);
        d.segd[s].count = n_live;
        d.segd[s].live = n_live;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.glob->cur_set ^= 1;
        d.glob->since_sort = 0u;  // the cell offsets are current
    }
}

// one block: the raw scan position of every segment, an exclusive prefix of
// the live counts in bin order (species-major, then instance)
__global__ __launch_bounds__(kBlock) void sort_start_kernel(Dev d)
{
    __shared__ unsigned long long s_w[kWaves];
    __shared__ unsigned long long s_carry;
    if (threadIdx.x == 0) s_carry = 0ull;
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    for (int base = 0; base < d.n_seg; base += kBlock) {
        const int q = base + threadIdx.x;  // position in bin order: q = sp * n_inst + inst
        int s = -1;
        unsigned long long v = 0ull;
        if (q < d.n_seg) {
            const int sp = q / d.n_inst, inst = q - sp * d.n_inst;
            s = inst * d.nsp + sp;
            v = d.segd[s].live;
        }
        unsigned long long inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned long long t = shfl_up_u64(inc, o);
            if (lane >= o) inc += t;
        }
        if (lane == 63) s_w[wave] = inc;
        __syncthreads();
        unsigned long long run = s_carry + inc - v;
        for (int w = 0; w < wave; ++w) run += s_w[w];
        if (s >= 0) {
            d.seg_start[s] = run;
            d.segd[s].vmax_bits = 0ull;
        }
        __syncthreads();
        if (threadIdx.x == kBlock - 1) s_carry = run + v;
        __syncthreads();
    }
}

hipError_t launch_sort(const Dev &d, hipStream_t st)
{
    const int grid = push_grid(d);
    if (d.precision == PIC_FP64)
        hipLaunchKernelGGL(sort_hist_kernel<true>, dim3(grid), dim3(kBlock), 0, st, d);
    else
        hipLaunchKernelGGL(sort_hist_kernel<false>, dim3(grid), dim3(kBlock), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_start_kernel, dim3(1), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scan_kernel, dim3((unsigned)d.n_sort_tiles), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (d.precision == PIC_FP64)
        hipLaunchKernelGGL(sort_scatter_kernel<true>, dim3(grid), dim3(kBlock), 0, st, d);
    else
        hipLaunchKernelGGL(sort_scatter_kernel<false>, dim3(grid), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_finish_kernel, dim3(1), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
