// init.hip -- the drawn initial state (PIC_INIT_DEVICE): every segment's
// n_init particles written into buffer set 0 from the counter-based
// generator, before the first step (gfx950).
//
// Particle p of species k of instance i: id = id0_k + p; Philox blocks
// (id, step -1, b = 0, 1) with the instance's key.  Position uniform (or a
// lattice), a pair copy of species 0's final position, an electron
// displacement (A/kk) sin(kk x) of mode m; velocity Maxwellian by
// Box-Muller.  Sec. 2: particles are initialised before the cycle starts.
#include "device_common.h"

#pragma clang fp contract(off)

namespace picx {

// position of particle p (id `id`) of a species of `kind` with `n` initial
// particles, in cells, inside [0, nc)
__device__ double init_position(const InstConst &ic, const SegConst &sc, int kind, int64_t p,
                                int64_t n, unsigned long long id)
{
    const double L = (double)ic.nc;
    double x;
    if (ic.init_opts & PIC_INIT_OPT_QUIET) {
        x = ((double)p + 0.5) * L / (double)n;
    } else {
        const uint4 u = draw(id, -1, 0, sc.key0, sc.key1);
        x = u01(u.x) * L;
    }
    if (ic.init_amp != 0.0 && kind == PIC_KIND_ELECTRON) {
        const double kk = 2.0 * M_PI * (double)ic.init_mode / L;
        x = x + (ic.init_amp / kk) * sin(kk * x);
        if (ic.bc == PIC_BC_PERIODIC) x = x - L * floor(x / L);
    }
    if (x >= L) x = nextafter(L, 0.0);
    if (x < 0.0) x = 0.0;
    return x;
}

__global__ __launch_bounds__(kBlock) void init_device_kernel(Dev d)
{
    const bool f64 = (d.precision == PIC_FP64);
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int seg = seg_of_tile(d.seg_tile0, d.n_seg, t);
        const SegConst &sc = d.segc[seg];
        const int64_t n = sc.n_init;
        const int64_t t0 = (t - sc.tile0) * (int64_t)kTile;
        if (t0 >= n) continue;
        const InstConst &ic = d.instc[sc.inst];
        const SegConst &s0 = d.segc[ic.seg0];
        const bool copy = (ic.init_opts & PIC_INIT_OPT_PAIR) && sc.sp > 0 && n == s0.n_init;
        for (int k = 0; k < kPer; ++k) {
            const int64_t p = t0 + (int64_t)(wave * kPer + k) * 64 + lane;
            if (p >= n) continue;
            const unsigned long long id = sc.id0 + (unsigned long long)p;
            const double x = copy ? init_position(ic, s0, s0.kind, p, n, s0.id0 + (unsigned long long)p)
                                  : init_position(ic, sc, sc.kind, p, n, id);
            const uint4 u = draw(id, -1, 0, sc.key0, sc.key1);
            const uint4 u1 = draw(id, -1, 1, sc.key0, sc.key1);
            double n0, n1, n2, n3;
            box_muller(u.y, u.z, n0, n1);
            box_muller(u.w, u1.x, n2, n3);
            const double vx = sc.vth_init * n0, vy = sc.vth_init * n1, vz = sc.vth_init * n2;
            const int64_t g = sc.base + p;
            if (f64) {
                ((double *)d.x[0])[g] = x;
                ((double *)d.vx[0])[g] = vx;
                ((double *)d.vy[0])[g] = vy;
                ((double *)d.vz[0])[g] = vz;
            } else {
                int32_t cell;
                float f;
                split_position(x, ic.nc, cell, f);
                d.cell[0][g] = cell;
                ((float *)d.x[0])[g] = f;
                ((float *)d.vx[0])[g] = (float)vx;
                ((float *)d.vy[0])[g] = (float)vy;
                ((float *)d.vz[0])[g] = (float)vz;
            }
            store_id(d, 0, g, id);
        }
    }
}

hipError_t launch_init_device(const Dev &d, hipStream_t st)
{
    hipLaunchKernelGGL(init_device_kernel, dim3(push_grid(d)), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace picx
