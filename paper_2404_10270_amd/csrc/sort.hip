// sort.hip -- "natural sorting" (paper Sec. 2: particles stored grouped by
// the cell they occupy) as a counting sort by cell into the other buffer set,
// dropping absorbed particles (gfx950).
//
//   hist     one bin per (species, node); absorbed particles go to the bin of
//            node nc, which no live particle uses; atomics pre-summed over
//            runs of equal cells in each wave
//   scan     single-pass exclusive scan of all bins (decoupled look-back);
//            writes the scatter cursors and the per-segment cell offsets
//   scatter  every live particle takes cursor[bin]++ (one atomic per run) and
//            is copied to its segment's region of the other set; the last
//            block switches the current set and sets the counts
#include "device_common.h"

namespace picx {

__device__ __forceinline__ int bin_of(const Dev &d, int cur, const SegConst &sc, int64_t g,
                                      bool f64, bool &live)
{
    int n;
    if (f64) {
        const double x = ((const double *)d.x[cur])[g];
        live = x >= 0.0;
        n = live ? (int)floor(x) : sc.nc;
    } else {
        const int32_t c = d.cell[cur][g];
        live = c >= 0;
        n = live ? c : sc.nc;
    }
    return (int)(sc.sp * d.G + sc.gnode + n);
}

__global__ __launch_bounds__(kBlock) void sort_hist_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            int key = -1;
            if (i < count) {
                bool live;
                key = bin_of(d, cur, sc, sc.base + i, f64, live);
            }
            bool tail;
            const unsigned long long s = run_sum(key, key >= 0 ? 1ull : 0ull, tail);
            if (tail && key >= 0) atomicAdd(d.hist + key, (uint32_t)s);
        }
    }
}

__device__ __forceinline__ unsigned long long ld_acq(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_rel(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// raw scan position of the first bin of segment `seg`: all occupied slots of
// the segments whose bins come earlier (bins are species-major, then instance)
__device__ unsigned long long seg_raw_start(const Dev &d, int seg)
{
    const SegConst &sc = d.segc[seg];
    unsigned long long s = 0;
    for (int q = 0; q < d.n_seg; ++q) {
        const SegConst &o = d.segc[q];
        if (o.sp < sc.sp || (o.sp == sc.sp && o.inst < sc.inst)) s += d.segd[q].count;
    }
    return s;
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
                    f = ld_acq(&st[p]);
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

template <typename T>
__device__ __forceinline__ void mv(void *dst, const void *src, int64_t to, int64_t from)
{
    ((T *)dst)[to] = ((const T *)src)[from];
}

__global__ __launch_bounds__(kBlock) void sort_scatter_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    const int nxt = cur ^ 1;
    const bool f64 = (d.precision == PIC_FP64);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        const unsigned long long start = d.seg_start[seg];
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            const int64_t g = sc.base + i;
            int key = -1;
            if (i < count) {
                bool live;
                key = bin_of(d, cur, sc, g, f64, live);
                if (!live) key = -1;
            }
            bool tail;
            const unsigned long long inc = run_sum(key, key >= 0 ? 1ull : 0ull, tail);
            const unsigned long long tails = ballot(tail);
            uint32_t base = 0;
            if (tail && key >= 0) base = atomicAdd(d.cursor + key, (uint32_t)inc);
            // every lane fetches the base of its run from the run's tail lane
            const unsigned long long above = tails & ~((1ull << lane) - 1ull);
            const int tl = __ffsll((long long)above) - 1;
            base = __shfl(base, tl, 64);
            if (key >= 0) {
                const uint32_t pos = base + (uint32_t)inc - 1u;
                const uint32_t rel = pos - (uint32_t)start;
                if (rel >= sc.cap) {  // cannot happen with a consistent histogram
                    atomicOr(&d.instd[sc.inst].status, PIC_ST_INTERNAL);
                    continue;
                }
                const int64_t to = sc.base + (int64_t)rel;
                if (f64) {
                    mv<double>(d.x[nxt], d.x[cur], to, g);
                    mv<double>(d.vx[nxt], d.vx[cur], to, g);
                    mv<double>(d.vy[nxt], d.vy[cur], to, g);
                    mv<double>(d.vz[nxt], d.vz[cur], to, g);
                } else {
                    mv<float>(d.x[nxt], d.x[cur], to, g);
                    mv<int32_t>(d.cell[nxt], d.cell[cur], to, g);
                    mv<float>(d.vx[nxt], d.vx[cur], to, g);
                    mv<float>(d.vy[nxt], d.vy[cur], to, g);
                    mv<float>(d.vz[nxt], d.vz[cur], to, g);
                }
                mv<unsigned long long>(d.id[nxt], d.id[cur], to, g);
            }
        }
    }
    // last block: switch sets and set the counts to the live particles
    __shared__ bool s_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(&d.glob->scatter_done, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    for (int s = threadIdx.x; s < d.n_seg; s += kBlock) {
        const SegConst &sc = d.segc[s];
        // offsets[node nc] of the segment = number of live particles
        const uint32_t n_live = d.offsets[sc.sp * d.G + sc.gnode + sc.nc];
        if (n_live != d.segd[s].live) atomicOr(&d.instd[sc.inst].status, PIC_ST_INTERNAL);
        d.segd[s].count = n_live;
        d.segd[s].live = n_live;
    }
    if (threadIdx.x == 0) {
        d.glob->cur_set = nxt;
        d.glob->scatter_done = 0;
    }
}

__global__ void sort_start_kernel(Dev d)
{
    for (int s = threadIdx.x; s < d.n_seg; s += blockDim.x) d.seg_start[s] = seg_raw_start(d, s);
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
    return hipGetLastError();
}

}  // namespace picx
