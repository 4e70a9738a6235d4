// push.hip -- the mover (paper Sec. 2, phase 5; moveb listing of Sec. 6) and
// the fixed-point charge deposition (Sec. 2, phase 1) for gfx950.
//
// One pass per particle and step: linear gather of the grid acceleration at
// the in-cell offset, magnetised Boris velocity update, advance x += vx,
// absorbing or periodic walls, the null-collision candidate test (one Philox
// block keyed by id and step), and the deposit of the new position.
//
// Layout: structure-of-arrays streamed once.  A block owns a tile of
// kTile consecutive slots of one segment; each wave takes kPer chunks of 64
// consecutive slots, so every load and store is a 256-byte (FP32) or
// 512-byte (FP64) coalesced access.  Cell-sorted neighbours deposit into the
// same nodes, so each chunk first sums its weights over runs of equal cells
// (wave-level segmented reduction) and only run tails issue the two 64-bit
// atomics.
#include "device_common.h"

#pragma clang fp contract(off)

namespace picx {

// deposit a chunk: lanes with key >= 0 add W1 = rint(f 2^32) to node key+1 and
// 2^32 - W1 to node key (linear weights, every particle adds exactly 2^32)
__device__ __forceinline__ void deposit_chunk(unsigned long long *__restrict__ S, int key,
                                              unsigned long long w1)
{
    // pack (count, sum W1): W1 <= 2^32 and at most 64 lanes -> sum < 2^39
    const unsigned long long v = (key >= 0) ? ((1ull << 40) + w1) : 0ull;
    bool tail;
    const unsigned long long t = run_sum(key, v, tail);
    if (tail && key >= 0) {
        const unsigned long long n = t >> 40;
        const unsigned long long b = t & ((1ull << 40) - 1ull);
        const unsigned long long a = (n << PIC_FRAC_BITS) - b;
        if (a) atomicAdd(S + key, a);
        if (b) atomicAdd(S + key + 1, b);
    }
}

// ---------------------------------------------------------------------------
// FP32 form: (int32 cell, float f in [0,1), float v), FP32 gather and push
// ---------------------------------------------------------------------------
template <bool DEP, bool MCC>
__global__ __launch_bounds__(kBlock) void push_f32_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    float *__restrict__ X = (float *)d.x[cur];
    int32_t *__restrict__ CELL = d.cell[cur];
    float *__restrict__ VX = (float *)d.vx[cur];
    float *__restrict__ VY = (float *)d.vy[cur];
    float *__restrict__ VZ = (float *)d.vz[cur];
    const unsigned long long *__restrict__ ID = d.id[cur];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;

    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        const float *__restrict__ acc = d.acc32 + sc.sp * d.G + sc.gnode;
        unsigned long long *__restrict__ S = d.S + sc.sp * d.G + sc.gnode;
        const int nc = sc.nc;
        const bool periodic = (sc.bc == PIC_BC_PERIODIC);
        const float tx = sc.txf, ty = sc.tyf, sx = sc.sxf, sy = sc.syf;
        long long step = 0;
        unsigned long long T = 0;
        if (MCC) {
            step = d.instd[sc.inst].step;
            T = sc.T;
        }
        SegDyn *sd = d.segd + seg;
        InstDyn *idn = d.instd + sc.inst;

#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            const bool valid = i < count;
            const int64_t g = sc.base + i;
            int32_t j = kDeadCell;
            if (valid) j = CELL[g];
            const bool live = valid && j >= 0;
            float f = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
            unsigned long long pid = 0;
            if (live) {
                f = X[g];
                vx = VX[g];
                vy = VY[g];
                vz = VZ[g];
                if (MCC) pid = ID[g];
            }
            bool left = false, right = false, bad = false, cfl = false, cand = false;
            int key = -1;
            unsigned long long w1 = 0;
            if (live) {
                // gather: a = a[j] + f (a[j+1] - a[j])
                const float a0 = acc[j], a1 = acc[j + 1];
                const float a = fmaf(f, a1 - a0, a0);
                const float h = 0.5f * a;
                const float mx = vx + h, my = vy, mz = vz;
                const float px = mx - mz * ty;
                const float py = my + mz * tx;
                const float pz = mz + (mx * ty - my * tx);
                const float qx = mx - pz * sy;
                const float qy = my + pz * sx;
                const float qz = mz + (px * sy - py * sx);
                vx = qx + h;
                vy = qy;
                vz = qz;
                // advance in cell-relative coordinates
                float fn = f + vx;
                // |fl| is clamped so that a runaway (flagged) particle still maps to a
                // valid integer cell
                const float fl = fminf(fmaxf(floorf(fn), -16777216.0f), 16777216.0f);
                fn = fn - fl;
                int32_t jn = j + (int32_t)fl;
                if (fn >= 1.0f) { fn = 0.0f; jn += 1; }
                cfl = !(fabsf(vx) < 1.0f);
                bad = !isfinite(vx) || !isfinite(vy) || !isfinite(vz);
                if (bad) jn = j, fn = f;  // keep the slot well-formed; the run is flagged
                if (periodic) {
                    if (jn < 0) jn += nc;
                    else if (jn >= nc) jn -= nc;
                    if (jn < 0 || jn >= nc) {
                        jn %= nc;
                        if (jn < 0) jn += nc;
                    }
                } else if (jn < 0) {
                    left = true;
                } else if (jn >= nc) {
                    right = true;
                }
                f = fn;
                j = (left || right) ? kDeadCell : jn;
                if (j >= 0) {
                    key = j;
                    w1 = (unsigned long long)rintf(f * 4294967296.0f);
                    if (MCC) {
                        const uint4 u = draw(pid, step, 0, sc.key0, sc.key1);
                        cand = (unsigned long long)u.x < T;
                    }
                }
                X[g] = f;
                CELL[g] = j;
                VX[g] = vx;
                VY[g] = vy;
                VZ[g] = vz;
            }
            wave_count(&sd->absorbed_step[0], left);
            wave_count(&sd->absorbed_step[1], right);
            wave_or(&idn->status, PIC_ST_CFL, cfl);
            wave_or(&idn->status, PIC_ST_NONFINITE, bad);
            if (MCC) {
                const uint32_t idx = wave_append(&d.glob->cand_count, cand);
                if (cand) {
                    if (idx < (uint32_t)d.cand_cap) d.cand[idx] = (uint32_t)g;
                    else atomicOr(&idn->status, PIC_ST_CANDIDATES);
                }
            }
            if (DEP) deposit_chunk(S, key, w1);
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 form: double x in cells, double v; the same arithmetic as the FP64
// reference, operation by operation (no contraction, explicit fma in the gather)
// ---------------------------------------------------------------------------
template <bool DEP, bool MCC>
__global__ __launch_bounds__(kBlock) void push_f64_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    double *__restrict__ X = (double *)d.x[cur];
    double *__restrict__ VX = (double *)d.vx[cur];
    double *__restrict__ VY = (double *)d.vy[cur];
    double *__restrict__ VZ = (double *)d.vz[cur];
    const unsigned long long *__restrict__ ID = d.id[cur];
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;

    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        const double *__restrict__ acc = d.acc64 + sc.sp * d.G + sc.gnode;
        unsigned long long *__restrict__ S = d.S + sc.sp * d.G + sc.gnode;
        const double L = (double)sc.nc;
        const bool periodic = (sc.bc == PIC_BC_PERIODIC);
        const double tx = sc.tx, ty = sc.ty, sx = sc.sx, sy = sc.sy;
        long long step = 0;
        unsigned long long T = 0;
        if (MCC) {
            step = d.instd[sc.inst].step;
            T = sc.T;
        }
        SegDyn *sd = d.segd + seg;
        InstDyn *idn = d.instd + sc.inst;

#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            const bool valid = i < count;
            const int64_t g = sc.base + i;
            double x = kDeadX;
            if (valid) x = X[g];
            const bool live = valid && x >= 0.0;
            double vx = 0.0, vy = 0.0, vz = 0.0;
            unsigned long long pid = 0;
            if (live) {
                vx = VX[g];
                vy = VY[g];
                vz = VZ[g];
                if (MCC) pid = ID[g];
            }
            bool left = false, right = false, bad = false, cfl = false, cand = false;
            int key = -1;
            unsigned long long w1 = 0;
            if (live) {
                const double jd = floor(x);
                const double f = x - jd;
                const int32_t j = (int32_t)jd;
                const double a = fma(f, acc[j + 1] - acc[j], acc[j]);
                const double h = 0.5 * a;
                const double mx = vx + h, my = vy, mz = vz;
                const double px = mx - mz * ty;
                const double py = my + mz * tx;
                const double pz = mz + (mx * ty - my * tx);
                const double qx = mx - pz * sy;
                const double qy = my + pz * sx;
                const double qz = mz + (px * sy - py * sx);
                vx = qx + h;
                vy = qy;
                vz = qz;
                double xn = x + vx;
                cfl = !(fabs(vx) < 1.0);
                bad = !isfinite(vx) || !isfinite(vy) || !isfinite(vz);
                if (bad) xn = x;
                if (periodic) {
                    if (xn < 0.0) xn += L;
                    else if (xn >= L) xn -= L;
                    if (xn >= L) xn -= L;
                    if (!(xn >= 0.0 && xn < L)) {  // displacement beyond one period (flagged)
                        xn = xn - L * floor(xn / L);
                        if (!(xn >= 0.0 && xn < L)) xn = 0.0;
                    }
                } else if (xn < 0.0) {
                    left = true;
                } else if (xn >= L) {
                    right = true;
                }
                x = (left || right) ? kDeadX : xn;
                if (x >= 0.0) {
                    const double jn = floor(x);
                    key = (int)jn;
                    w1 = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
                    if (MCC) {
                        const uint4 u = draw(pid, step, 0, sc.key0, sc.key1);
                        cand = (unsigned long long)u.x < T;
                    }
                }
                X[g] = x;
                VX[g] = vx;
                VY[g] = vy;
                VZ[g] = vz;
            }
            wave_count(&sd->absorbed_step[0], left);
            wave_count(&sd->absorbed_step[1], right);
            wave_or(&idn->status, PIC_ST_CFL, cfl);
            wave_or(&idn->status, PIC_ST_NONFINITE, bad);
            if (MCC) {
                const uint32_t idx = wave_append(&d.glob->cand_count, cand);
                if (cand) {
                    if (idx < (uint32_t)d.cand_cap) d.cand[idx] = (uint32_t)g;
                    else atomicOr(&idn->status, PIC_ST_CANDIDATES);
                }
            }
            if (DEP) deposit_chunk(S, key, w1);
        }
    }
}

// ---------------------------------------------------------------------------
// standalone deposit of the current positions (both forms)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void deposit_kernel(Dev d)
{
    const int cur = d.glob->cur_set;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const bool f64 = (d.precision == PIC_FP64);
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t count = d.segd[seg].count;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= count) continue;
        unsigned long long *__restrict__ S = d.S + sc.sp * d.G + sc.gnode;
        for (int k = 0; k < kPer; ++k) {
            const int64_t i = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            const int64_t g = sc.base + i;
            int key = -1;
            unsigned long long w1 = 0;
            if (i < count) {
                if (f64) {
                    const double x = ((const double *)d.x[cur])[g];
                    if (x >= 0.0) {
                        const double jn = floor(x);
                        key = (int)jn;
                        w1 = (unsigned long long)rint(ldexp(x - jn, PIC_FRAC_BITS));
                    }
                } else {
                    const int32_t j = d.cell[cur][g];
                    if (j >= 0) {
                        key = j;
                        w1 = (unsigned long long)rintf(((const float *)d.x[cur])[g] * 4294967296.0f);
                    }
                }
            }
            deposit_chunk(S, key, w1);
        }
    }
}

int push_grid(const Dev &d)
{
    // persistent-style grid: enough blocks to fill 256 CUs several times over,
    // never more than there are tiles
    int64_t g = d.n_tiles;
    const int64_t cap = 256 * 16;
    if (g > cap) g = cap;
    if (g < 1) g = 1;
    return (int)g;
}

hipError_t launch_push(const Dev &d, hipStream_t st, bool dep, bool mcc)
{
    const dim3 grid(push_grid(d)), block(kBlock);
    if (d.precision == PIC_FP64) {
        if (dep && mcc) hipLaunchKernelGGL((push_f64_kernel<true, true>), grid, block, 0, st, d);
        else if (dep) hipLaunchKernelGGL((push_f64_kernel<true, false>), grid, block, 0, st, d);
        else if (mcc) hipLaunchKernelGGL((push_f64_kernel<false, true>), grid, block, 0, st, d);
        else hipLaunchKernelGGL((push_f64_kernel<false, false>), grid, block, 0, st, d);
    } else {
        if (dep && mcc) hipLaunchKernelGGL((push_f32_kernel<true, true>), grid, block, 0, st, d);
        else if (dep) hipLaunchKernelGGL((push_f32_kernel<true, false>), grid, block, 0, st, d);
        else if (mcc) hipLaunchKernelGGL((push_f32_kernel<false, true>), grid, block, 0, st, d);
        else hipLaunchKernelGGL((push_f32_kernel<false, false>), grid, block, 0, st, d);
    }
    return hipGetLastError();
}

hipError_t launch_deposit(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(deposit_kernel, dim3(push_grid(d)), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
