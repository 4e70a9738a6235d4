// layout.hip -- libpic_layout: the FP32 mover pass of libpic over one
// species with the particles stored in four layouts (pic_layout.h), for the
// layout study that arXiv 2404.10270 proposes (Sec. 6: vector-of-structs and
// array-of-structs movers; Sec. 2: particles kept grouped by cell).
//
// Every layout runs the same per-particle arithmetic as libpic's FP32 mover
// (gather fma(f, a1 - a0, a0), half kick, Boris rotation, half kick,
// advance, periodic re-entry, the candidate draw of Philox block (id, step,
// 0)) and the same deposit through per-wave LDS windows (mover_common.h), on
// the same persistent grid of 1024-slot tiles; only where the particle
// fields live differs:
//   SOA      six arrays (libpic);
//   AOS      one 32-byte struct per particle, read as two 16-byte loads;
//   AOSOA    64-particle blocks with the six arrays inside each block;
//   CELLPAD  `slack` slots per cell and a count per cell; the cell is
//            implicit in the slot, so 24 B are read and 16 B + the id are
//            written per particle, but every pass regroups the particles by
//            cell into the other buffer (per-wave reservations in the
//            destination cells).
#include <vector>

#include "mover_common.h"
#include "pic_layout.h"

#pragma clang fp contract(off)

namespace picx {
namespace {

constexpr int kPerL = 4;                 // 64-slot chunks per wave per tile
constexpr int kTileL = kBlock * kPerL;   // slots per tile
constexpr int kGridL = 2048;             // persistent grid
constexpr uint64_t kHeader = 256 + sizeof(unsigned long long) * kGridL;  // status + candidate partials

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct AosP {
    int32_t cell;
    float f, vx, vy, vz;
    uint32_t pad;
    unsigned long long id;
};
static_assert(sizeof(AosP) == 32, "AoS record is 32 bytes");

struct AosoaB {
    int32_t cell[64];
    float f[64], vx[64], vy[64], vz[64];
    unsigned long long id[64];
};

uint64_t align256(uint64_t v) { return (v + 255u) & ~uint64_t(255); }

// pointers into the work buffer of one layout
struct View {
    uint32_t *status;
    unsigned long long *cand_part;   // [kGridL]
    // SOA
    int32_t *cell;
    float *f, *vx, *vy, *vz;
    unsigned long long *id;
    // AOS, AOSOA
    AosP *aos;
    AosoaB *blk;
    // CELLPAD: two buffers, counts and the offsets of pls_store
    float *cf[2], *cvx[2], *cvy[2], *cvz[2];
    unsigned long long *cid[2];
    uint32_t *cnt[2];
    int64_t *off;
    int64_t n_slots;  // slots the move kernel walks
    uint64_t bytes;
};

View make_view(int layout, int64_t n, int32_t nc, int32_t slack, void *work)
{
    View v{};
    char *w = (char *)work;
    uint64_t o = 0;
    auto take = [&](uint64_t b) {
        const uint64_t r = o;
        o = align256(o + b);
        return w ? w + r : nullptr;
    };
    v.status = (uint32_t *)take(256);
    v.cand_part = (unsigned long long *)take(sizeof(unsigned long long) * kGridL);
    const uint64_t un = (uint64_t)n;
    if (layout == PLS_SOA) {
        v.cell = (int32_t *)take(4 * un);
        v.f = (float *)take(4 * un);
        v.vx = (float *)take(4 * un);
        v.vy = (float *)take(4 * un);
        v.vz = (float *)take(4 * un);
        v.id = (unsigned long long *)take(8 * un);
        v.n_slots = n;
    } else if (layout == PLS_AOS) {
        v.aos = (AosP *)take(sizeof(AosP) * un);
        v.n_slots = n;
    } else if (layout == PLS_AOSOA) {
        const uint64_t nb = (un + 63) / 64;
        v.blk = (AosoaB *)take(sizeof(AosoaB) * nb);
        v.n_slots = (int64_t)nb * 64;
    } else {
        const uint64_t ns = (uint64_t)nc * (uint64_t)slack;
        for (int b = 0; b < 2; ++b) {
            v.cf[b] = (float *)take(4 * ns);
            v.cvx[b] = (float *)take(4 * ns);
            v.cvy[b] = (float *)take(4 * ns);
            v.cvz[b] = (float *)take(4 * ns);
            v.cid[b] = (unsigned long long *)take(8 * ns);
            v.cnt[b] = (uint32_t *)take(4 * (uint64_t)nc);
        }
        v.off = (int64_t *)take(8 * (uint64_t)nc);
        v.n_slots = (int64_t)ns;
    }
    v.bytes = o;
    return v;
}

struct Args {
    View v;
    pls_params p;
    long long step;
    int rd;   // CELLPAD: buffer read by this pass
};

// one particle's push (libpic's FP32 mover with nstep = 1, periodic)
__device__ __forceinline__ void move_one(const pls_params &p, float a0, float a1, int32_t &j, float &f,
                                         float &vx, float &vy, float &vz)
{
    const float a = fmaf(f, a1 - a0, a0);
    const float h = 0.5f * a;
    const float mx = vx + h, my = vy, mz = vz;
    const float px = mx - mz * p.ty;
    const float py = my + mz * p.tx;
    const float pz = mz + (mx * p.ty - my * p.tx);
    const float qx = mx - pz * p.sy;
    const float qy = my + pz * p.sx;
    const float qz = mz + (px * p.sy - py * p.sx);
    const float nvx = qx + h;
    float fn = f + 1.0f * nvx;
    const float fl = fminf(fmaxf(floorf(fn), -16777216.0f), 16777216.0f);
    fn = fn - fl;
    int32_t jn = j + (int32_t)fl;
    if (fn >= 1.0f) {
        fn = 0.0f;
        jn += 1;
    }
    const int nc = p.nc;
    if (jn < 0) jn += nc;
    else if (jn >= nc) jn -= nc;
    if (jn < 0 || jn >= nc) {
        jn %= nc;
        if (jn < 0) jn += nc;
    }
    j = jn;
    f = fn;
    vx = nvx;
    vy = qy;
    vz = qz;
}

template <int L>
__global__ __launch_bounds__(kBlock) void move_kernel(Args a)
{
    __shared__ unsigned long long wdep[kWaves][kWaveWin];  // each wave's deposit window
    __shared__ unsigned long long s_cand[kWaves];
    for (int i = threadIdx.x; i < kWaves * kWaveWin; i += kBlock) (&wdep[0][0])[i] = 0ull;
    __syncthreads();
    const View &v = a.v;
    const pls_params &p = a.p;
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int64_t n_tiles = (v.n_slots + kTileL - 1) / kTileL;
    const int slack = p.slack;
    const int rd = a.rd, wr = a.rd ^ 1;
    uint32_t n_cand = 0;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        int32_t j[kPerL];
        float f[kPerL], vx[kPerL], vy[kPerL], vz[kPerL];
        unsigned long long id[kPerL];
        // one chunk of the tile (slot s, lane's part), in the layout
        auto load_chunk = [&](int k, int64_t s) {
            if (L == PLS_SOA) {
                j[k] = stream_ld(&v.cell[s]);
                f[k] = stream_ld(&v.f[s]);
                vx[k] = stream_ld(&v.vx[s]);
                vy[k] = stream_ld(&v.vy[s]);
                vz[k] = stream_ld(&v.vz[s]);
                id[k] = stream_ld(&v.id[s]);
            } else if (L == PLS_AOS) {
                const u32x4 lo = stream_ld((const u32x4 *)&v.aos[s]);
                const u32x4 hi = stream_ld((const u32x4 *)&v.aos[s] + 1);
                j[k] = (int32_t)lo.x;
                f[k] = __uint_as_float(lo.y);
                vx[k] = __uint_as_float(lo.z);
                vy[k] = __uint_as_float(lo.w);
                vz[k] = __uint_as_float(hi.x);
                id[k] = ((unsigned long long)hi.w << 32) | hi.z;
            } else if (L == PLS_AOSOA) {
                const AosoaB &b = v.blk[s >> 6];
                j[k] = stream_ld(&b.cell[lane]);
                f[k] = stream_ld(&b.f[lane]);
                vx[k] = stream_ld(&b.vx[lane]);
                vy[k] = stream_ld(&b.vy[lane]);
                vz[k] = stream_ld(&b.vz[lane]);
                id[k] = stream_ld(&b.id[lane]);
            } else {
                const int64_t c = s / slack;
                const int64_t r = s - c * slack;
                if (r < (int64_t)v.cnt[rd][c]) {
                    j[k] = (int32_t)c;
                    f[k] = stream_ld(&v.cf[rd][s]);
                    vx[k] = stream_ld(&v.cvx[rd][s]);
                    vy[k] = stream_ld(&v.cvy[rd][s]);
                    vz[k] = stream_ld(&v.cvz[rd][s]);
                    id[k] = stream_ld(&v.cid[rd][s]);
                }
            }
        };
        // the three flat layouts load unpredicated (a lane past the end
        // reads the last slot again and is marked empty after all loads), so
        // the wave issues every load before its first wait
#pragma unroll
        for (int k = 0; k < kPerL; ++k) {
            const int64_t s = t * kTileL + (int64_t)(wave * kPerL + k) * 64 + lane;
            j[k] = -1;
            f[k] = vx[k] = vy[k] = vz[k] = 0.f;
            id[k] = 0;
            if (L != PLS_CELLPAD) load_chunk(k, s < v.n_slots ? s : v.n_slots - 1);
            else if (s < v.n_slots) load_chunk(k, s);
        }
        if (L != PLS_CELLPAD) {
#pragma unroll
            for (int k = 0; k < kPerL; ++k)
                if (t * kTileL + (int64_t)(wave * kPerL + k) * 64 + lane >= v.n_slots) j[k] = -1;
        }
        // the gather unpredicated (an empty slot reads node 0 and ignores it)
        float a0[kPerL], a1[kPerL];
#pragma unroll
        for (int k = 0; k < kPerL; ++k) {
            const int jj = j[k] >= 0 ? j[k] : 0;
            a0[k] = p.acc[jj];
            a1[k] = p.acc[jj + 1];
        }
        int key[kPerL];
        unsigned long long w1[kPerL];
        bool live[kPerL];
#pragma unroll
        for (int k = 0; k < kPerL; ++k) {
            live[k] = j[k] >= 0;
            key[k] = -1;
            w1[k] = 0;
            if (!live[k]) continue;
            move_one(p, a0[k], a1[k], j[k], f[k], vx[k], vy[k], vz[k]);
            key[k] = j[k];
            w1[k] = (unsigned long long)rintf(f[k] * 4294967296.0f);
            const uint4 u = draw(id[k], a.step, 0, p.key0, p.key1);
            n_cand += ((unsigned long long)u.x < p.T) ? 1u : 0u;
        }
#pragma unroll
        for (int k = 0; k < kPerL; ++k) {
            const int64_t s = t * kTileL + (int64_t)(wave * kPerL + k) * 64 + lane;
            if (L == PLS_CELLPAD) {
                // reserve slots in the destination cell, one atomic per run of equal cells
                bool tail;
                const unsigned long long inc = run_sum(key[k], live[k] ? 1ull : 0ull, tail);
                const unsigned long long tails = ballot(tail);
                uint32_t base = 0;
                if (tail && live[k]) base = atomicAdd(&v.cnt[wr][key[k]], (uint32_t)inc);
                const unsigned long long above = tails & ~((1ull << lane) - 1ull);
                const int tl = __ffsll((long long)above) - 1;
                base = __shfl(base, tl, 64);
                if (!live[k]) continue;
                const uint32_t r = base + (uint32_t)inc - 1u;
                if (r >= (uint32_t)slack) {
                    atomicOr(v.status, 1u);
                    continue;
                }
                const int64_t d = (int64_t)key[k] * slack + r;
                stream_st(&v.cf[wr][d], f[k]);
                stream_st(&v.cvx[wr][d], vx[k]);
                stream_st(&v.cvy[wr][d], vy[k]);
                stream_st(&v.cvz[wr][d], vz[k]);
                stream_st(&v.cid[wr][d], id[k]);
                continue;
            }
            if (!live[k]) continue;
            if (L == PLS_SOA) {
                stream_st(&v.cell[s], j[k]);
                stream_st(&v.f[s], f[k]);
                stream_st(&v.vx[s], vx[k]);
                stream_st(&v.vy[s], vy[k]);
                stream_st(&v.vz[s], vz[k]);
            } else if (L == PLS_AOS) {
                u32x4 lo;
                lo.x = (uint32_t)j[k];
                lo.y = __float_as_uint(f[k]);
                lo.z = __float_as_uint(vx[k]);
                lo.w = __float_as_uint(vy[k]);
                stream_st((u32x4 *)&v.aos[s], lo);
                stream_st(&v.aos[s].vz, vz[k]);
            } else {
                AosoaB &b = v.blk[s >> 6];
                stream_st(&b.cell[lane], j[k]);
                stream_st(&b.f[lane], f[k]);
                stream_st(&b.vx[lane], vx[k]);
                stream_st(&b.vy[lane], vy[k]);
                stream_st(&b.vz[lane], vz[k]);
            }
        }
        deposit_wave<kPerL>(wdep[wave], (unsigned long long *)p.S, key, w1);
    }
    // this block's candidates into its own slot
    uint32_t c = n_cand;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += (uint32_t)__shfl_xor((int)c, o, 64);
    if (lane == 0) s_cand[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += s_cand[w];
        v.cand_part[blockIdx.x] += tot;
    }
}

__global__ void clear_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void pack_kernel(int layout, View v, pls_soa in, int64_t n, int32_t slack)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (layout == PLS_AOSOA && i < v.n_slots && i >= n) v.blk[i >> 6].cell[i & 63] = -1;
    if (i >= n) return;
    const int32_t c = in.cell[i];
    if (layout == PLS_AOS) {
        AosP r;
        r.cell = c;
        r.f = in.f[i];
        r.vx = in.vx[i];
        r.vy = in.vy[i];
        r.vz = in.vz[i];
        r.pad = 0u;
        r.id = in.id[i];
        v.aos[i] = r;
    } else if (layout == PLS_AOSOA) {
        AosoaB &b = v.blk[i >> 6];
        const int q = (int)(i & 63);
        b.cell[q] = c;
        b.f[q] = in.f[i];
        b.vx[q] = in.vx[i];
        b.vy[q] = in.vy[i];
        b.vz[q] = in.vz[i];
        b.id[q] = in.id[i];
    } else {
        const uint32_t r = atomicAdd(&v.cnt[0][c], 1u);
        if (r >= (uint32_t)slack) {
            atomicOr(v.status, 1u);
            return;
        }
        const int64_t d = (int64_t)c * slack + r;
        v.cf[0][d] = in.f[i];
        v.cvx[0][d] = in.vx[i];
        v.cvy[0][d] = in.vy[i];
        v.cvz[0][d] = in.vz[i];
        v.cid[0][d] = in.id[i];
    }
}

__global__ void unpack_kernel(int layout, View v, pls_soa out, int64_t n, int32_t slack, int buf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (layout == PLS_CELLPAD) {
        if (i >= v.n_slots) return;
        const int64_t c = i / slack, r = i - c * slack;
        if (r >= (int64_t)v.cnt[buf][c]) return;
        const int64_t o = v.off[c] + r;
        out.cell[o] = (int32_t)c;
        out.f[o] = v.cf[buf][i];
        out.vx[o] = v.cvx[buf][i];
        out.vy[o] = v.cvy[buf][i];
        out.vz[o] = v.cvz[buf][i];
        out.id[o] = v.cid[buf][i];
        return;
    }
    if (i >= n) return;
    if (layout == PLS_AOS) {
        const AosP r = v.aos[i];
        out.cell[i] = r.cell;
        out.f[i] = r.f;
        out.vx[i] = r.vx;
        out.vy[i] = r.vy;
        out.vz[i] = r.vz;
        out.id[i] = r.id;
    } else {
        const AosoaB &b = v.blk[i >> 6];
        const int q = (int)(i & 63);
        out.cell[i] = b.cell[q];
        out.f[i] = b.f[q];
        out.vx[i] = b.vx[q];
        out.vy[i] = b.vy[q];
        out.vz[i] = b.vz[q];
        out.id[i] = b.id[q];
    }
}

bool valid_layout(int layout) { return layout >= 0 && layout < PLS_N_LAYOUTS; }

bool valid_sizes(int layout, int64_t n, int32_t nc, int32_t slack)
{
    if (n < 0 || n > ((int64_t)1 << 31) || nc < 2) return false;
    if (layout == PLS_CELLPAD && (slack < 64 || slack % 64 != 0 || (int64_t)nc * slack > ((int64_t)1 << 31)))
        return false;
    return true;
}

int grid_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace
}  // namespace picx

using namespace picx;

extern "C" {

int pls_work_bytes(int layout, int64_t n, int32_t nc, int32_t slack, uint64_t *bytes)
{
    if (!bytes || !valid_layout(layout) || !valid_sizes(layout, n, nc, slack)) return -1;
    *bytes = make_view(layout, n, nc, slack, nullptr).bytes;
    return 0;
}

int pls_load(int layout, const pls_soa *in, int64_t n, int32_t nc, int32_t slack, void *work,
             void *stream)
{
    if (!in || !work || !valid_layout(layout) || !valid_sizes(layout, n, nc, slack)) return -1;
    hipStream_t st = (hipStream_t)stream;
    const View v = make_view(layout, n, nc, slack, work);
    bool ok = hipMemsetAsync(work, 0, kHeader, st) == hipSuccess;
    if (layout == PLS_SOA) {
        ok = ok && hipMemcpyAsync(v.cell, in->cell, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(v.f, in->f, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(v.vx, in->vx, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(v.vy, in->vy, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(v.vz, in->vz, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(v.id, in->id, 8 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        return ok ? 0 : -3;
    }
    if (layout == PLS_CELLPAD) ok = ok && hipMemsetAsync(v.cnt[0], 0, 4 * (size_t)nc, st) == hipSuccess;
    const int64_t m = layout == PLS_AOSOA ? v.n_slots : n;
    if (ok && m > 0) {
        hipLaunchKernelGGL(pack_kernel, dim3(grid_for(m)), dim3(kBlock), 0, st, layout, v, *in, n,
                           slack);
        ok = hipGetLastError() == hipSuccess;
    }
    return ok ? 0 : -3;
}

int pls_step(int layout, const pls_params *p, int64_t n, int64_t pass, int64_t step, void *work,
             void *stream)
{
    if (!p || !work || !p->acc || !p->S || !valid_layout(layout) ||
        !valid_sizes(layout, n, p->nc, p->slack) || pass < 0)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    Args a;
    a.v = make_view(layout, n, p->nc, p->slack, work);
    a.p = *p;
    a.step = (long long)step;
    a.rd = (int)(pass & 1);
    if (layout == PLS_CELLPAD) {
        hipLaunchKernelGGL(clear_u32, dim3(256), dim3(kBlock), 0, st, a.v.cnt[a.rd ^ 1], (int64_t)p->nc);
        if (hipGetLastError() != hipSuccess) return -3;
    }
    const dim3 grid(kGridL), block(kBlock);
    switch (layout) {
    case PLS_SOA: hipLaunchKernelGGL(move_kernel<PLS_SOA>, grid, block, 0, st, a); break;
    case PLS_AOS: hipLaunchKernelGGL(move_kernel<PLS_AOS>, grid, block, 0, st, a); break;
    case PLS_AOSOA: hipLaunchKernelGGL(move_kernel<PLS_AOSOA>, grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL(move_kernel<PLS_CELLPAD>, grid, block, 0, st, a); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int pls_store(int layout, void *work, int64_t n, int32_t nc, int32_t slack, int64_t passes,
              pls_soa *out, int64_t *n_out, uint64_t *n_cand, void *stream)
{
    if (!out || !work || !n_out || !n_cand || !valid_layout(layout) ||
        !valid_sizes(layout, n, nc, slack) || passes < 0)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    const View v = make_view(layout, n, nc, slack, work);
    const int buf = (int)(passes & 1);
    int64_t m = n;
    bool ok = true;
    if (layout == PLS_SOA) {
        ok = ok && hipMemcpyAsync(out->cell, v.cell, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(out->f, v.f, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(out->vx, v.vx, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(out->vy, v.vy, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(out->vz, v.vz, 4 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
        ok = ok && hipMemcpyAsync(out->id, v.id, 8 * n, hipMemcpyDeviceToDevice, st) == hipSuccess;
    } else if (layout == PLS_CELLPAD) {
        // the offsets of the cells from their counts (on the host; not timed)
        std::vector<uint32_t> cnt((size_t)nc);
        std::vector<int64_t> off((size_t)nc);
        ok = hipMemcpyAsync(cnt.data(), v.cnt[buf], 4 * (size_t)nc, hipMemcpyDeviceToHost, st) == hipSuccess;
        ok = ok && hipStreamSynchronize(st) == hipSuccess;
        int64_t run = 0;
        for (int32_t c = 0; c < nc; ++c) {
            off[(size_t)c] = run;
            run += cnt[(size_t)c];
        }
        m = run;
        if (m > n) return -1;  // the caller's output holds n particles
        ok = ok && hipMemcpyAsync(v.off, off.data(), 8 * (size_t)nc, hipMemcpyHostToDevice, st) == hipSuccess;
        if (ok && v.n_slots > 0) {
            hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(v.n_slots)), dim3(kBlock), 0, st, layout, v,
                               *out, n, slack, buf);
            ok = hipGetLastError() == hipSuccess;
        }
        ok = ok && hipStreamSynchronize(st) == hipSuccess;  // off must outlive the copy
    } else if (n > 0) {
        hipLaunchKernelGGL(unpack_kernel, dim3(grid_for(n)), dim3(kBlock), 0, st, layout, v, *out, n,
                           slack, buf);
        ok = hipGetLastError() == hipSuccess;
    }
    uint32_t status = 0;
    std::vector<unsigned long long> part(kGridL);
    ok = ok && hipMemcpyAsync(&status, v.status, 4, hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipMemcpyAsync(part.data(), v.cand_part, sizeof(unsigned long long) * kGridL,
                              hipMemcpyDeviceToHost, st) == hipSuccess;
    ok = ok && hipStreamSynchronize(st) == hipSuccess;
    if (!ok) return -3;
    uint64_t c = 0;
    for (unsigned long long q : part) c += q;
    *n_cand = c;
    *n_out = m;
    return status ? -4 : 0;
}

}  // extern "C"
