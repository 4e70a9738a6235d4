// step_close.h -- the event index of a step and the close of the step
// (counts, ids, wall-loss totals, step index), shared by the collision
// kernels and the field solve, whose first launch can close the step in one
// block of its own.
#pragma once

#include "device_common.h"

namespace picx {

// ---------------------------------------------------------------------------
// the event list of this step: per-block regions indexed by an LDS prefix sum
// ---------------------------------------------------------------------------
struct EventIndex {
    uint32_t pre[kMaxPushBlocks + 1];
    uint32_t in_regions, total;
};

// builds the prefix over the regions (all threads; barriers inside)
__device__ inline void build_event_index(EventIndex &X, const Dev &d)
{
    const int nb = d.n_push_blocks;
    constexpr int kPerT = (kMaxPushBlocks + kBlock - 1) / kBlock;
    uint32_t v[kPerT];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int b = threadIdx.x * kPerT + r;
        v[r] = (b < nb) ? d.ev_n[b] : 0u;
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
        const int b = threadIdx.x * kPerT + r;
        if (b <= nb) X.pre[b] = run;
        run += v[r];
    }
    if (threadIdx.x == kBlock - 1) {
        uint32_t ovf = d.glob->ev_ovf;
        if (ovf > (uint32_t)d.ev_ovf_cap) ovf = (uint32_t)d.ev_ovf_cap;
        X.in_regions = run;
        X.total = run + ovf;
        if (nb == kMaxPushBlocks) X.pre[nb] = run;
    }
    __syncthreads();
}

// the index index_kernel wrote, into LDS (all threads; a barrier inside)
__device__ inline void load_event_index(EventIndex &X, const Dev &d)
{
    // all of a thread's loads before its first LDS store (unpredicated: an
    // index past the last region reads the last entry again)
    constexpr int kPerT = (kMaxPushBlocks + 1 + kBlock - 1) / kBlock;
    const int nb = d.n_push_blocks;
    uint32_t v[kPerT];
#pragma unroll
    for (int r = 0; r < kPerT; ++r) v[r] = d.ev_pre[min(threadIdx.x + r * kBlock, (unsigned)nb)];
#pragma unroll
    for (int r = 0; r < kPerT; ++r) {
        const int b = threadIdx.x + r * kBlock;
        if (b <= nb) X.pre[b] = v[r];
    }
    if (threadIdx.x == 0) {
        X.total = d.glob->ev_total;
        X.in_regions = d.glob->ev_in_regions;
    }
    __syncthreads();
}

// the step's event index: a batch reads the one index_kernel wrote (its
// bucket kernels need the total before they start); a single instance builds
// it in every block (cheaper than a kernel of its own)
__device__ inline void get_event_index(EventIndex &X, const Dev &d)
{
    if (d.n_inst > 1) load_event_index(X, d);
    else build_event_index(X, d);
}

constexpr int kMaxInstLds = 4096;

// per-instance ionisation counts of this step (into LDS)
__device__ inline void count_events(const EventIndex &X, const Dev &d, uint32_t *s_m, int n_inst)
{
    if (d.n_inst == 1) {
        // a single instance owns every event
        if (threadIdx.x == 0) s_m[0] = X.total;
        __syncthreads();
        return;
    }
    // a batch: the bucket scan of this step holds the counts (it runs
    // whenever there are events and more than one instance)
    for (int i = threadIdx.x; i < n_inst; i += kBlock)
        s_m[i] = X.total ? d.inst_start[i + 1] - d.inst_start[i] : 0u;
    __syncthreads();
}

// ions lost to the walls this step = source pairs of the instance
__device__ __forceinline__ uint32_t source_pairs(const Dev &d, int i)
{
    const InstConst &ic = d.instc[i];
    if (!ic.source_on || ic.seg_i < 0) return 0u;
    return d.segd[ic.seg_i].absorbed_step[0] + d.segd[ic.seg_i].absorbed_step[1];
}

// close of the step (one block, all threads): counts, ids, wall-loss
// totals, step index, and the per-step lists cleared
__device__ inline void close_body(const Dev &d, const EventIndex &X, const uint32_t *s_m, int n_inst,
                           bool with_events)
{
    for (int i = threadIdx.x; i < d.n_inst; i += kBlock) {
        const InstConst &ic = d.instc[i];
        InstDyn *idn = d.instd + i;
        const uint32_t n_src = source_pairs(d, i);
        const uint32_t m_i = i < n_inst ? s_m[i] : 0u;
        unsigned long long pushed = 0;
        for (int k = 0; k < ic.nsp; ++k) {
            const int s = ic.seg0 + k;
            SegDyn *sd = d.segd + s;
            const SegConst &sc = d.segc[s];
            if (idn->step % sc.nstep == 0) pushed += sd->live;  // a subcycled species moved this step
            uint32_t requested = 0;
            if (s == ic.seg_e || s == ic.seg_i) requested = m_i + n_src;
            uint64_t n_new = (uint64_t)sd->count + requested;
            if (n_new > sc.cap) n_new = sc.cap;
            // created = the slots below capacity that were filled
            const uint32_t created = (uint32_t)(n_new - sd->count);
            const uint32_t lost = sd->absorbed_step[0] + sd->absorbed_step[1] + sd->consumed_step;
            sd->count = (uint32_t)n_new;
            sd->live = sd->live - lost + created;
            sd->consumed_step = 0;
            sd->absorbed_total[0] += sd->absorbed_step[0];
            sd->absorbed_total[1] += sd->absorbed_step[1];
            sd->created_total += created;
            sd->absorbed_step[0] = 0;
            sd->absorbed_step[1] = 0;
        }
        idn->particle_steps += pushed;
        idn->next_id += 2ull * (unsigned long long)(m_i + n_src);
        if (idn->next_id > (1ull << 32)) idn->wide_ids = 1u;  // ids created from now on may need id_hi
        idn->n_source += n_src;
        idn->step += 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        d.glob->cand_ovf = 0;
        d.glob->ev_ovf = 0;
        const uint32_t s = d.glob->since_sort;
        if (s != kNoIndex && s < kNoIndex - 1u) d.glob->since_sort = s + 1u;
    }
    // ranks back to zero for the next step
    if (with_events)
        for (uint32_t e = threadIdx.x; e < X.total; e += kBlock) {
            d.ev_rank[e] = 0u;
            d.ev_crank[e] = 0u;
        }
    // empty event regions for a step without collisions
    if (!with_events)
        for (int b = threadIdx.x; b < d.n_push_blocks; b += kBlock) d.ev_n[b] = 0u;
}

// with_events: 0 no collisions this step; 1 collisions, ranks in the rank
// array (cleared here); 2 a single instance whose emit kernel ranked its
// events itself and left their count in glob->ev_total (nothing to clear)
__device__ inline void close_step(const Dev &d, int with_events)
{
    __shared__ EventIndex X;
    __shared__ uint32_t s_m[kMaxInstLds];
    const int n_inst = d.n_inst < kMaxInstLds ? d.n_inst : kMaxInstLds;
    if (with_events == 2) {
        if (threadIdx.x == 0) {
            X.total = 0u;  // no ranks to clear
            s_m[0] = d.glob->ev_total;
        }
        __syncthreads();
        close_body(d, X, s_m, n_inst, true);
        return;
    }
    if (with_events) {
        get_event_index(X, d);
        count_events(X, d, s_m, n_inst);
    } else {
        if (threadIdx.x == 0) X.total = 0u;
        for (int i = threadIdx.x; i < n_inst; i += kBlock) s_m[i] = 0u;
        __syncthreads();
    }
    close_body(d, X, s_m, n_inst, with_events != 0);
}

}  // namespace picx
