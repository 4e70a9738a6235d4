// collide_common.h -- the collision of listed candidates (paper Sec. 2,
// phase 4: Monte Carlo collisions and ionisation), shared by the collide
// kernel and the movers that collide their own block's candidates right
// after their push (the block's candidate region is complete once its waves
// pass a barrier; no other block reads or writes it).
#pragma once

#include "device_common.h"

namespace picx {

__device__ __forceinline__ void st_v(void *p, int64_t g, double v, bool f64)
{
    if (f64) ((double *)p)[g] = v;
    else ((float *)p)[g] = (float)v;
}

// segments whose constants the collide kernel stages in LDS (few segments:
// a single instance or a small batch)
constexpr int kCollSegLds = 8;

// collide one listed candidate; returns its segment, fills the counts and
// the ionisation event, and stores the velocity of a particle that collided.
// SEGLDS: the segment constants and instance steps come from the block's LDS
// copies s_sc / s_step (staged at block start, beside the first loads).
template <bool SEGLDS>
__device__ __forceinline__ int collide_one(const Dev &d, int cur, bool f64, const Cand &c,
                                           const SegConst *s_sc, const long long *s_step,
                                           uint32_t &cnt, bool &iz, IzEvent &ev)
{
    const int64_t g = c.g;
    const int seg = c.seg;  // the mover's segment of the candidate
    const SegConst &sc = SEGLDS ? s_sc[seg] : d.segc[seg];
    const long long step = SEGLDS ? s_step[seg] : d.instd[sc.inst].step;
    double vx = c.vx, vy = c.vy, vz = c.vz;
    double g2 = 0.0;
    // with kinetic neutrals: the atom density at the electron (the mover's
    // linear weights on the node densities of the last field pass)
    int32_t cell = 0;
    Rates R;
    if (sc.kinetic) {
        double f;
        if (f64) {
            const double x = ((const double *)d.x[cur])[g];
            const double jd = floor(x);
            cell = (int32_t)jd;
            f = x - jd;
        } else {
            cell = d.cell[cur][g];
            f = (double)((const float *)d.x[cur])[g];
        }
        const double *nn = d.nn + sc.gnode;
        const double nl = fma(f, nn[cell + 1] - nn[cell], nn[cell]);
        if (nl > sc.n_bound) atomicOr(&d.instd[sc.inst].status, PIC_ST_NN_CAP);
        R = local_rates(sc, nl);
    } else {
        R = uniform_rates(sc);
    }
    collide_vel(sc, R, step, c.pid, vx, vy, vz, cnt, iz, g2);
    if (cnt & ((1u << kCEl) | (1u << kCIz) | (1u << kCCx) | (1u << kCEx))) {
        st_v(d.vx[cur], g, vx, f64);
        st_v(d.vy[cur], g, vy, f64);
        st_v(d.vz[cur], g, vz, f64);
    }
    if (iz) {
        ev.parent_id = c.pid;
        ev.slot = (uint32_t)g;
        ev.seg = seg;
        ev.inst = sc.inst;
        ev.cell = cell;
        ev.g2 = g2;
    }
    return seg;
}

__device__ __forceinline__ void add_counts(InstDyn *idn, uint32_t c)
{
    if (c & (1u << kCCand)) atomicAdd(&idn->n_candidates, 1ull);
    if (c & (1u << kCEl)) atomicAdd(&idn->n_elastic, 1ull);
    if (c & (1u << kCIz)) atomicAdd(&idn->n_ionize, 1ull);
    if (c & (1u << kCCx)) atomicAdd(&idn->n_cx, 1ull);
    if (c & (1u << kCOver)) atomicAdd(&idn->n_over_cap, 1ull);
    if (c & (1u << kCEx)) atomicAdd(&idn->n_excite, 1ull);
}

// The collisions of listed candidates by one block (all threads; barriers
// inside).  REGION: the block's own region `slot` of the candidate list (the
// counts of its wave parts in wave_n[kWaves], or cand_n when null), whose
// ionisation events go to event region `slot` (the excess to the event
// overflow list), and ev_n[slot] is written.  OVF: the block's share of the
// shared candidate overflow list among gridDim.x blocks; without REGION its
// events all go to the event overflow list.  Process counts go to count slot
// `slot` through s_cnt (LDS scratch of n_seg x kNCnt words, when lds_cnt) or
// to the instance totals.  s_sc / s_step: LDS copies of the segment
// constants and steps (SEGLDS, at most kCollSegLds segments).
template <bool SEGLDS>
__device__ void collide_block(const Dev &d, int slot, bool region, bool ovf, const uint32_t *wave_n,
                              uint32_t *s_cnt, bool lds_cnt, uint32_t &s_en, SegConst *s_sc,
                              long long *s_step)
{
    if (lds_cnt)
        for (int q = threadIdx.x; q < d.n_seg * kNCnt; q += kBlock) s_cnt[q] = 0u;
    if (threadIdx.x == 0) s_en = 0u;
    if (SEGLDS) {
        // the segments' constants word by word, and each segment's step
        constexpr int kW = (int)(sizeof(SegConst) / 8);
        static_assert(sizeof(SegConst) % 8 == 0, "segment constants: whole words");
        const unsigned long long *src = (const unsigned long long *)d.segc;
        unsigned long long *dst = (unsigned long long *)s_sc;
        for (int q = threadIdx.x; q < d.n_seg * kW; q += kBlock) dst[q] = src[q];
        if (threadIdx.x < d.n_seg) s_step[threadIdx.x] = d.instd[d.segc[threadIdx.x].inst].step;
    }
    __syncthreads();

    const int cur = d.glob->cur_set;
    const bool f64 = (d.precision == PIC_FP64);
    // the region (one part per mover wave), then a share of the overflow list
    const uint32_t qw = (uint32_t)d.cand_q / kWaves;
    uint32_t pre[kWaves + 1];
    pre[0] = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        pre[w + 1] = pre[w] + (region ? (wave_n ? wave_n[w] : d.cand_n[slot * kWaves + w]) : 0u);
    const uint32_t nr = pre[kWaves];
    uint32_t o_lo = 0, o_hi = 0;
    if (ovf) {
        uint32_t novf = d.glob->cand_ovf;
        if (novf > (uint32_t)d.cand_ovf_cap) novf = (uint32_t)d.cand_ovf_cap;
        const uint32_t per_block = (novf + gridDim.x - 1) / gridDim.x;
        o_lo = min(novf, blockIdx.x * per_block);
        o_hi = min(novf, o_lo + per_block);
    }
    const uint32_t n_items = nr + (o_hi - o_lo);
    // item q's entry: the region's wave parts, then the overflow share
    auto entry = [&](uint32_t q) -> int64_t {
        if (q < nr) {
            int w = 0;
#pragma unroll
            for (int v = 1; v < kWaves; ++v) w += (q >= pre[v]) ? 1 : 0;
            return (int64_t)slot * d.cand_q + (int64_t)w * qw + (q - pre[w]);
        }
        return (int64_t)d.n_regions * d.cand_q + o_lo + (q - nr);
    };
    // each candidate's entry is loaded while the thread's previous one is
    // collided (the loads would otherwise wait behind its stores)
    Cand cn{};
    if (threadIdx.x < n_items) cn = d.cand[entry(threadIdx.x)];
    for (uint32_t q = threadIdx.x; q < n_items; q += kBlock) {
        const Cand c = cn;
        if (q + kBlock < n_items) cn = d.cand[entry(q + kBlock)];
        uint32_t cnt = 0;  // one bit per process (1 << kC...)
        bool iz = false;
        IzEvent ev = {};
        const int seg = collide_one<SEGLDS>(d, cur, f64, c, s_sc, s_step, cnt, iz, ev);
        if (iz) {
            // this block's region of the event list; the rare excess goes to the overflow list
            const uint32_t e = region ? atomicAdd(&s_en, 1u) : (uint32_t)d.ev_q;
            if (e < (uint32_t)d.ev_q) {
                d.ev[(int64_t)slot * d.ev_q + e] = ev;
            } else {
                const uint32_t o = atomicAdd(&d.glob->ev_ovf, 1u);
                if (o < (uint32_t)d.ev_ovf_cap) d.ev[(int64_t)d.n_regions * d.ev_q + o] = ev;
                else atomicOr(&d.instd[ev.inst].status, PIC_ST_CANDIDATES);
            }
        }
        if (lds_cnt) {
#pragma unroll
            for (int c = 0; c < kNCnt; ++c)
                if (cnt & (1u << c)) atomicAdd(&s_cnt[seg * kNCnt + c], 1u);
        } else {
            add_counts(d.instd + d.segc[seg].inst, cnt);
        }
    }
    __syncthreads();
    if (region && threadIdx.x == 0) d.ev_n[slot] = min(s_en, (uint32_t)d.ev_q);
    if (lds_cnt) {
        // this block's own slot (no other block touches it), by atomics that
        // return nothing, so that the block does not wait for a read of it
        unsigned long long *cs = d.cnt_slot + (int64_t)slot * d.n_seg * kNCnt;
        for (int q = threadIdx.x; q < d.n_seg * kNCnt; q += kBlock) {
            const uint32_t v = s_cnt[q];
            if (v) atomicAdd(cs + q, (unsigned long long)v);
        }
    }
}

}  // namespace picx
