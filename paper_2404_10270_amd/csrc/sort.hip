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

// node of a slot, -1 when absorbed
__device__ __forceinline__ int node_of(const Dev &d, int cur, int64_t g, bool f64)
{
    if (f64) {
        const double x = ((const double *)d.x[cur])[g];
        return x >= 0.0 ? (int)floor(x) : -1;
    }
    return d.cell[cur][g];
}

// the keys of this wave's kPer chunks of the tile at slot base + t0 (-1 past
// count or absorbed).  A full tile loads unpredicated, with the precision
// branch outside the chunk loop, so the wave issues every load before one
// wait rather than waiting inside each chunk's branch.
__device__ __forceinline__ void tile_keys(const Dev &d, int cur, int64_t base, int64_t t0, int64_t count,
                                          bool f64, int (&key)[kPer])
{
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    if (t0 + kTile <= count) {
        const int64_t g0 = base + t0 + (int64_t)(wave * kPer) * 64 + lane;
        if (f64) {
            const double *X = (const double *)d.x[cur] + g0;
            double x[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) x[k] = __builtin_nontemporal_load(&X[k * 64]);
#pragma unroll
            for (int k = 0; k < kPer; ++k) key[k] = x[k] >= 0.0 ? (int)floor(x[k]) : -1;
        } else {
            const int32_t *CELL = d.cell[cur] + g0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) key[k] = __builtin_nontemporal_load(&CELL[k * 64]);
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
        key[k] = (i < count) ? node_of(d, cur, base + i, f64) : -1;
    }
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
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmn = min(kmn, __shfl_xor(kmn, o, 64));
        kmx = max(kmx, __shfl_xor(kmx, o, 64));
    }
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

__global__ __launch_bounds__(kBlock) void sort_hist_kernel(Dev d)
{
    __shared__ SortLds L;
    __shared__ uint32_t wcnt[kWaves][kHistWaveWin];  // each wave's window of bins
    for (int i = threadIdx.x; i < kWaves * kHistWaveWin; i += kBlock) (&wcnt[0][0])[i] = 0u;
    sort_lds_init(L, d);
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    uint32_t *W = wcnt[wave];
    int hint = 0;  // segment of the previous tile
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        int64_t tile0, base, count;
        const int seg = sort_tile_seg(L, d, t, tile0, base, count, hint);
        const int64_t t0 = (t - tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        const SegConst &sc = d.segc[seg];
        uint32_t *__restrict__ H = d.hist + sc.sp * d.G + sc.gnode;
        int key[kPer];
        tile_keys(d, cur, base, t0, count, f64, key);
        // this wave's bins: run sums of equal keys into its own LDS window (no
        // block barrier), then one global atomic per touched bin
        int kmn = 0x7fffffff, kmx = -1;
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (key[k] >= 0) {
                kmn = min(kmn, key[k]);
                kmx = max(kmx, key[k]);
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            kmn = min(kmn, __shfl_xor(kmn, o, 64));
            kmx = max(kmx, __shfl_xor(kmx, o, 64));
        }
        const int lo = __builtin_amdgcn_readfirstlane(kmn);
        const int hi = __builtin_amdgcn_readfirstlane(kmx);
        if (hi < 0) continue;  // no live particle in the wave's chunks
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            bool tail;
            const unsigned long long n = run_sum(key[k], key[k] >= 0 ? 1ull : 0ull, tail);
            if (tail && key[k] >= 0) {
                const int rel = key[k] - lo;
                if (rel < kHistWaveWin) atomicAdd(&W[rel], (uint32_t)n);
                else atomicAdd(H + key[k], (uint32_t)n);
            }
        }
        hist_wave_sync();
        const int span = min(hi - lo + 1, kHistWaveWin);
        for (int i = lane; i < span; i += 64) {
            const uint32_t v = W[i];
            if (v) {
                atomicAdd(H + lo + i, v);
                W[i] = 0u;
            }
        }
        hist_wave_sync();
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

// copy the fields of a wave's kPer chunks (slot g0 + 64 k) to slots to[k]
// (-1: none) of the other set: all loads, then all stores
template <typename V, bool CELL>
__device__ __forceinline__ void move_fields(const Dev &d, int cur, int nxt, int64_t g0,
                                            const int64_t (&to)[kPer], bool full)
{
    V x[kPer], vx[kPer], vy[kPer], vz[kPer];
    int32_t c[kPer];
    unsigned long long id[kPer];
    const V *X = (const V *)d.x[cur], *VX = (const V *)d.vx[cur], *VY = (const V *)d.vy[cur],
            *VZ = (const V *)d.vz[cur];
    // the source arrays are streamed once per sort: nontemporal loads keep
    // them from displacing the bins, cursors and the scattered destinations
    // in L2 (the stores stay cached: a tile's particles go to many bins, and
    // L2 merges their partial lines)
    auto load = [&](int k) {
        const int64_t g = g0 + (int64_t)k * 64;
        x[k] = __builtin_nontemporal_load(&X[g]);
        vx[k] = __builtin_nontemporal_load(&VX[g]);
        vy[k] = __builtin_nontemporal_load(&VY[g]);
        vz[k] = __builtin_nontemporal_load(&VZ[g]);
        if (CELL) c[k] = __builtin_nontemporal_load(&d.cell[cur][g]);
        id[k] = (unsigned long long)__builtin_nontemporal_load(&d.id_lo[cur][g]) |
                ((unsigned long long)__builtin_nontemporal_load(&d.id_hi[cur][g]) << 32);
    };
    if (full) {
        // every slot of a full tile exists: its loads go unpredicated (an
        // absorbed particle's fields are read and not stored)
#pragma unroll
        for (int k = 0; k < kPer; ++k) load(k);
    } else {
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (to[k] >= 0) load(k);
    }
    V *Xn = (V *)d.x[nxt], *VXn = (V *)d.vx[nxt], *VYn = (V *)d.vy[nxt], *VZn = (V *)d.vz[nxt];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        if (to[k] < 0) continue;
        const int64_t t = to[k];
        Xn[t] = x[k];
        VXn[t] = vx[k];
        VYn[t] = vy[k];
        VZn[t] = vz[k];
        if (CELL) d.cell[nxt][t] = c[k];
        store_id(d, nxt, t, id[k]);
    }
}

__global__ __launch_bounds__(kBlock) void sort_scatter_kernel(Dev d)
{
    __shared__ SortLds L;
    sort_lds_init(L, d);
    const int cur = d.glob->cur_set;
    const int nxt = cur ^ 1;
    const bool f64 = (d.precision == PIC_FP64);
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
        const SegConst &sc = d.segc[seg];
        const uint32_t start = (uint32_t)d.seg_start[seg];
        uint32_t *__restrict__ CUR = d.cursor + sc.sp * d.G + sc.gnode;
        int key[kPer];
        tile_keys(d, cur, base, t0, count, f64, key);
        if (w0) tile_grab(Q);  // the next tile, behind this one's key loads
        int lo, hi;
        tile_window(L, key, lo, hi);
        // rank of every particle among the tile's particles of its cell
        uint32_t rank[kPer];
        bool outside[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            bool tail;
            const unsigned long long inc = run_sum(key[k], key[k] >= 0 ? 1ull : 0ull, tail);
            const unsigned long long tails = ballot(tail);
            const int rel = key[k] - lo;
            outside[k] = key[k] >= 0 && rel >= kSortWin;
            uint32_t rb = 0;
            if (tail && key[k] >= 0) {
                // in-window bins: rank within the tile; outside: a direct global reservation
                if (!outside[k]) rb = atomicAdd(&L.cnt[rel], (uint32_t)inc);
                else rb = atomicAdd(CUR + key[k], (uint32_t)inc);
            }
            const unsigned long long above = tails & ~((1ull << lane) - 1ull);
            const int tl = __ffsll((long long)above) - 1;
            rb = __shfl(rb, tl, 64);
            rank[k] = rb + (uint32_t)inc - 1u;
        }
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
        // destinations; then every field of the tile's particles is loaded
        // before any is stored (a store to the other set could alias a later
        // load in the compiler's view, which would otherwise keep each load
        // waiting behind the previous store)
        // (the segment's cap and base read once: the status atomic below would
        // otherwise make the compiler read them again, with a wait, per chunk)
        const uint32_t cap = sc.cap;
        const int64_t sbase = sc.base;
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
        const int64_t g0 = base + t0 + (int64_t)(wave * kPer) * 64 + lane;
        const bool full = t0 + kTile <= count;
        if (f64) {
            move_fields<double, false>(d, cur, nxt, g0, to, full);
        } else {
            move_fields<float, true>(d, cur, nxt, g0, to, full);
        }
        if (sc.kind == PIC_KIND_NEUTRAL) {
            unsigned long long vb = 0ull;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                if (key[k] < 0) continue;
                const int64_t g = base + t0 + (int64_t)(wave * kPer + k) * 64 + lane;
                const double v = f64 ? fabs(((const double *)d.vx[cur])[g])
                                     : fabs((double)((const float *)d.vx[cur])[g]);
                const unsigned long long b = (unsigned long long)__double_as_longlong(v);
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
    hipLaunchKernelGGL(sort_hist_kernel, dim3(grid), dim3(kBlock), 0, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_start_kernel, dim3(1), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scan_kernel, dim3((unsigned)d.n_sort_tiles), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_scatter_kernel, dim3(grid), dim3(kBlock), 0, st, d);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sort_finish_kernel, dim3(1), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
