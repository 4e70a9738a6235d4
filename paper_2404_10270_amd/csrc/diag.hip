// diag.hip -- diagnostics (FP64 moments per species and instance) and the
// validation of an uploaded initial state (gfx950).
#include "device_common.h"

namespace picx {

// per-block partial sums: [block][segment][kDiagVals]; the block processes a
// fixed set of tiles, so the partials depend only on the particle order
__global__ __launch_bounds__(kBlock) void diag_partial_kernel(Dev d)
{
    extern __shared__ double s_acc[];  // [n_seg][kDiagVals]
    __shared__ double s_red[kDiagVals][kBlock];
    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    for (int q = threadIdx.x; q < d.n_seg * kDiagVals; q += kBlock) s_acc[q] = 0.0;
    __syncthreads();
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        double a[kDiagVals] = {0, 0, 0, 0, 0, 0};
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            if (i >= count) continue;
            const int64_t g = sc.base + i;
            bool live;
            double vx, vy, vz;
            if (f64) {
                live = ((const double *)d.x[cur])[g] >= 0.0;
                vx = ((const double *)d.vx[cur])[g];
                vy = ((const double *)d.vy[cur])[g];
                vz = ((const double *)d.vz[cur])[g];
            } else {
                live = d.cell[cur][g] >= 0;
                vx = ((const float *)d.vx[cur])[g];
                vy = ((const float *)d.vy[cur])[g];
                vz = ((const float *)d.vz[cur])[g];
            }
            if (!live) continue;
            a[0] += 1.0;
            a[1] += (vx * vx + vy * vy) + vz * vz;
            a[2] += vx;
            a[3] += vy;
            a[4] += vz;
        }
        for (int v = 0; v < kDiagVals; ++v) s_red[v][threadIdx.x] = a[v];
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s)
                for (int v = 0; v < kDiagVals; ++v) s_red[v][threadIdx.x] += s_red[v][threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x < kDiagVals) s_acc[seg * kDiagVals + threadIdx.x] += s_red[threadIdx.x][0];
        __syncthreads();
    }
    double *out = d.diag_part + (int64_t)blockIdx.x * d.n_seg * kDiagVals;
    for (int q = threadIdx.x; q < d.n_seg * kDiagVals; q += kBlock) out[q] = s_acc[q];
}

// block-wide sum in a fixed order (deterministic)
__device__ double block_sum(double v, double *s_red)
{
    s_red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) s_red[threadIdx.x] += s_red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = s_red[0];
    __syncthreads();
    return r;
}

// one block per instance: sums of the per-block partials, the process-count
// slots and the field-energy tiles
__global__ __launch_bounds__(kBlock) void diag_final_kernel(Dev d, int n_blocks)
{
    __shared__ double s_red[kBlock];
    const int i = blockIdx.x;
    const InstConst &ic = d.instc[i];
    const InstDyn &idn = d.instd[i];
    double mom[PIC_MAX_SPECIES][kDiagVals];
    for (int k = 0; k < ic.nsp; ++k) {
        const int s = ic.seg0 + k;
        for (int v = 0; v < kDiagVals; ++v) {
            double a = 0.0;
            for (int b = threadIdx.x; b < n_blocks; b += kBlock)
                a += d.diag_part[((int64_t)b * d.n_seg + s) * kDiagVals + v];
            mom[k][v] = block_sum(a, s_red);
        }
    }
    unsigned long long pc[kNCnt] = {idn.n_candidates, idn.n_elastic, idn.n_ionize, idn.n_cx,
                                    idn.n_over_cap, idn.n_excite};
    if (d.n_seg <= kCntSegMax) {
        for (int q = 0; q < kNCnt; ++q) {
            double a = 0.0;  // exact: counts stay far below 2^53
            for (int b = threadIdx.x; b < d.n_regions; b += kBlock)
                for (int k = 0; k < ic.nsp; ++k)
                    a += (double)d.cnt_slot[((int64_t)b * d.n_seg + ic.seg0 + k) * kNCnt + q];
            pc[q] += (unsigned long long)block_sum(a, s_red);
        }
    }
    double fe = 0.0;
    for (int64_t t = ic.ftile0 + threadIdx.x; t < d.inst_ftile0[i + 1]; t += kBlock) fe += d.fe_part[t];
    fe = block_sum(fe, s_red);
    if (threadIdx.x != 0) return;
    pic_diag o;
    memset(&o, 0, sizeof(o));
    o.step = idn.step;
    o.next_id = idn.next_id;
    o.status = idn.status;
    o.cur_set = d.glob->cur_set;
    for (int k = 0; k < ic.nsp; ++k) {
        const int s = ic.seg0 + k;
        const SegConst &sc = d.segc[s];
        const SegDyn &sd = d.segd[s];
        o.n_slots_used[k] = sd.count;
        o.n_live[k] = (int64_t)mom[k][0];
        o.ke[k] = 0.5 * sc.mw * (sc.vs * sc.vs) * mom[k][1];
        o.mom[k][0] = sc.mw * sc.vs * mom[k][2];
        o.mom[k][1] = sc.mw * sc.vs * mom[k][3];
        o.mom[k][2] = sc.mw * sc.vs * mom[k][4];
        o.absorbed_total[k][0] = (int64_t)sd.absorbed_total[0];
        o.absorbed_total[k][1] = (int64_t)sd.absorbed_total[1];
        o.created_total[k] = (int64_t)sd.created_total;
    }
    o.field_energy = 0.5 * ic.eps0 * fe;
    o.n_candidates = (int64_t)pc[0];
    o.n_elastic = (int64_t)pc[1];
    o.n_ionize = (int64_t)pc[2];
    o.n_cx = (int64_t)pc[3];
    o.n_over_cap = (int64_t)pc[4];
    o.n_excite = (int64_t)pc[5];
    o.n_consumed = (int64_t)idn.n_consumed;
    o.n_iz_untargeted = (int64_t)idn.n_iz_untargeted;
    o.n_source = (int64_t)idn.n_source;
    o.particle_steps = (int64_t)idn.particle_steps;
    d.diag_out[i] = o;
}

int diag_blocks(const Dev &d)
{
    int64_t g = d.n_tiles;
    if (g > kDiagBlocks) g = kDiagBlocks;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_diag(const Dev &d, hipStream_t st)
{
    const int nb = diag_blocks(d);
    const size_t lds = (size_t)d.n_seg * kDiagVals * sizeof(double);
    hipLaunchKernelGGL(diag_partial_kernel, dim3(nb), dim3(kBlock), lds, st, d);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(d.n_inst), dim3(kBlock), 0, st, d, nb);
    return hipGetLastError();
}

// uploaded state: a particle outside [0, nc), with a position offset outside
// [0, 1) or a non-finite velocity is dropped (marked absorbed) and flagged;
// an id at or above 2^32 marks its instance's ids as wide
__global__ __launch_bounds__(kBlock) void init_check_kernel(Dev d)
{
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
            bool drop = false;
            if (i < count) {
                const int64_t g = sc.base + i;
                if (f64) {
                    const double x = ((const double *)d.x[0])[g];
                    const double vx = ((const double *)d.vx[0])[g];
                    const double vy = ((const double *)d.vy[0])[g];
                    const double vz = ((const double *)d.vz[0])[g];
                    drop = !(x >= 0.0 && x < (double)sc.nc) || !isfinite(vx) || !isfinite(vy) ||
                           !isfinite(vz);
                    if (drop) ((double *)d.x[0])[g] = kDeadX;
                } else {
                    const int32_t c = d.cell[0][g];
                    const float f = ((const float *)d.x[0])[g];
                    const float vx = ((const float *)d.vx[0])[g];
                    const float vy = ((const float *)d.vy[0])[g];
                    const float vz = ((const float *)d.vz[0])[g];
                    drop = !(c >= 0 && c < sc.nc) || !(f >= 0.0f && f < 1.0f) || !isfinite(vx) ||
                           !isfinite(vy) || !isfinite(vz);
                    if (drop) d.cell[0][g] = kDeadCell;
                }
            }
            const bool wide = i < count && d.id_hi[0][sc.base + i] != 0u;
            const unsigned long long m = ballot(drop);
            if (m && lane == (__ffsll((long long)m) - 1)) {
                atomicSub(&d.segd[seg].live, (uint32_t)__popcll(m));
                atomicOr(&d.instd[sc.inst].status, PIC_ST_BAD_INIT);
            }
            // an uploaded id at or above 2^32: the movers read both id words
            const unsigned long long mw = ballot(wide);
            if (mw && lane == (__ffsll((long long)mw) - 1)) atomicOr(&d.instd[sc.inst].wide_ids, 1u);
        }
    }
}

hipError_t launch_init_state(const Dev &d, hipStream_t st, const uint32_t *)
{
    hipLaunchKernelGGL(init_check_kernel, dim3(push_grid(d)), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
