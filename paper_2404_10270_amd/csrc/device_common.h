// device_common.h -- wave64 utilities, the counter-based generator and small
// helpers shared by libpic's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#include "pic_internal.h"

namespace picx {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies by fixed odd constants whose halves are mixed with
// the other two counter words and the key; the key advances by the two Weyl
// constants after every round.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
        const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
        c = make_uint4(n0, (uint32_t)p1, n2, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// draw block b of particle `id` at `step`
__device__ __forceinline__ uint4 draw(unsigned long long id, long long step, uint32_t b,
                                      uint32_t k0, uint32_t k1)
{
    return philox(make_uint4((uint32_t)id, (uint32_t)(id >> 32), (uint32_t)step, b), k0, k1);
}

// draw block b of source pair k at `step` (counter word 1 = 0xFFFFFFFF, never an id's)
__device__ __forceinline__ uint4 draw_source(unsigned long long k, long long step, uint32_t b,
                                             uint32_t k0, uint32_t k1)
{
    return philox(make_uint4((uint32_t)k, 0xFFFFFFFFu, (uint32_t)step, b), k0, k1);
}

// uniform on (0,1): (u + 1/2) 2^-32, exact in FP64
__device__ __forceinline__ double u01(uint32_t u) { return ((double)u + 0.5) * 0x1p-32; }

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }

// Wave-wide minimum and maximum of a signed int through DPP lane moves (no
// LDS round trip): within each row of 16 lanes by the xor-1 and xor-2 quad
// permutes and the half-row and row mirrors, then across rows by the row
// broadcasts of lanes 15 and 31, which leave the result in lane 63.
constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror
constexpr int kDppBcast15 = 0x142;    // row_bcast:15 (rows 1 and 3 take lane 15 of the row before)
constexpr int kDppBcast31 = 0x143;    // row_bcast:31 (rows 2 and 3 take lane 31)

template <bool MAX, int CTRL, int ROWS>
__device__ __forceinline__ int dpp_step(int v)
{
    const int ident = MAX ? INT_MIN : INT_MAX;
    const int o = __builtin_amdgcn_update_dpp(ident, v, CTRL, ROWS, 0xF, false);
    return MAX ? max(v, o) : min(v, o);
}

template <bool MAX>
__device__ __forceinline__ int wave_reduce_dpp(int v)
{
    v = dpp_step<MAX, kDppQuadXor1, 0xF>(v);
    v = dpp_step<MAX, kDppQuadXor2, 0xF>(v);
    v = dpp_step<MAX, kDppHalfMirror, 0xF>(v);
    v = dpp_step<MAX, kDppMirror, 0xF>(v);
    v = dpp_step<MAX, kDppBcast15, 0xA>(v);
    v = dpp_step<MAX, kDppBcast31, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, int d)
{
    const uint32_t lo = __shfl_up((uint32_t)v, d, 64);
    const uint32_t hi = __shfl_up((uint32_t)(v >> 32), d, 64);
    return ((unsigned long long)hi << 32) | lo;
}

// Reduction over runs of equal keys in lane order.  Every lane passes a key
// and a value; a run is a maximal group of consecutive lanes with equal
// keys.  On return, the last lane of each run has is_tail = true and holds
// the run's sum (other lanes hold partial sums).  Used to pre-aggregate
// atomics when neighbouring lanes target the same address (cell-sorted
// particles).
__device__ __forceinline__ unsigned long long run_sum(int key, unsigned long long v,
                                                      bool &is_tail)
{
    const int lane = lane_id();
    const int up = __shfl_up(key, 1, 64);
    const int dn = __shfl_down(key, 1, 64);
    const bool head = (lane == 0) || (up != key);
    is_tail = (lane == 63) || (dn != key);
    const unsigned long long heads = ballot(head);
    // index of this lane's run head: highest set bit of heads at or below lane
    const unsigned long long mask = heads & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
    const int h = 63 - __clzll(mask);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long o = shfl_up_u64(v, d);
        if (lane - d >= h) v += o;
    }
    return v;
}

// wave-aggregated append: every lane with `pred` gets a unique index from
// *counter; returns the index (undefined where !pred)
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred)
{
    const unsigned long long m = ballot(pred);
    uint32_t base = 0;
    const int lane = lane_id();
    const int leader = m ? (__ffsll((long long)m) - 1) : 0;
    if (m && lane == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader, 64);
    const unsigned long long below = m & ((1ull << lane) - 1ull);
    return base + (uint32_t)__popcll(below);
}

// wave-aggregated add of a per-lane 0/1 flag to a counter (one atomic per wave)
__device__ __forceinline__ void wave_count(uint32_t *counter, bool pred)
{
    const unsigned long long m = ballot(pred);
    if (m && lane_id() == (__ffsll((long long)m) - 1)) atomicAdd(counter, (uint32_t)__popcll(m));
}

__device__ __forceinline__ void wave_or(uint32_t *word, uint32_t bits, bool pred)
{
    const unsigned long long m = ballot(pred);
    if (m && lane_id() == (__ffsll((long long)m) - 1)) atomicOr(word, bits);
}

// segment owning virtual tile t (binary search in tile0[0..n_seg])
__device__ __forceinline__ int seg_of_tile(const int64_t *tile0, int n_seg, int64_t t)
{
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// segment owning global slot g (binary search in seg_base[0..n_seg])
__device__ __forceinline__ int seg_of_slot(const int64_t *base, int n_seg, int64_t g)
{
    int lo = 0, hi = n_seg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// isotropic unit vector: cos(chi) = 1 - 2U, phi = 2 pi U'
__device__ __forceinline__ void iso_dir(uint32_t a, uint32_t b, double &d0, double &d1,
                                        double &d2)
{
    const double cc = 1.0 - 2.0 * u01(a);
    const double ss = sqrt(fmax(0.0, 1.0 - cc * cc));
    const double ph = 2.0 * M_PI * u01(b);
    double sp, cp;
    sincos(ph, &sp, &cp);
    d0 = cc;
    d1 = ss * cp;
    d2 = ss * sp;
}

// Box-Muller pair of standard normals
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, double &n0, double &n1)
{
    const double r = sqrt(-2.0 * log(u01(a)));
    const double t = 2.0 * M_PI * u01(b);
    double st, ct;
    sincos(t, &st, &ct);
    n0 = r * ct;
    n1 = r * st;
}

// ---------------------------------------------------------------------------
// Null-collision Monte Carlo for one candidate (Vahedi & Surendra, CPC 87,
// 1995).  The candidate's first Philox block (id, step, 0) is redrawn;
// r = U(u1) nu_max is compared, in FP64 and squared form, with the cumulative
// (n sigma_k dx) |v| of the processes in a fixed order:
//   electron  elastic (cold neutral of mass M, isotropic in the centre of
//             mass); excitation above its threshold (loses E_ex, isotropic);
//             ionisation above its threshold (energy above it split U : 1-U,
//             the first electron isotropic; the second electron's speed is
//             returned in g2 for the pair creation), its slot n sig_iz dx
//             |v|, or n sig_iz dx v_cap with a constant rate coefficient;
//   ion       charge exchange (the ion takes a Maxwellian velocity at T_n).
// n is the uniform gas density, or the local density of kinetic neutrals.
// (vx, vy, vz) in cells/step are updated in place; ev gets one bit per
// process that happened (1 << kC...; a candidate sets each bit at most once).
// ---------------------------------------------------------------------------
enum { kCCand = 0, kCEl = 1, kCIz = 2, kCCx = 3, kCOver = 4, kCEx = 5 };

// squares of the cumulative (n sigma) dx, and the constant-rate ionisation slot
struct Rates {
    double C0, C1, C2, crate;
};

__device__ __forceinline__ Rates uniform_rates(const SegConst &sc)
{
    return Rates{sc.C0, sc.C1, sc.C2, sc.crate};
}

// an electron's rates at the local neutral density nl [m^-3]
__device__ __forceinline__ Rates local_rates(const SegConst &sc, double nl)
{
    const double c0 = (nl * sc.sig_el) * sc.dxm;
    const double c1 = (nl * (sc.sig_el + sc.sig_ex)) * sc.dxm;
    const double c2 = (nl * ((sc.sig_el + sc.sig_ex) + sc.sig_iz)) * sc.dxm;
    return Rates{c0 * c0, c1 * c1, c2 * c2, ((nl * sc.sig_iz) * sc.dxm) * sc.vcap_hat};
}

__device__ __forceinline__ void collide_vel(const SegConst &sc, const Rates &R, long long step,
                                            unsigned long long pid, double &vx, double &vy,
                                            double &vz, uint32_t &ev, bool &iz, double &g2)
{
    const uint4 u = draw(pid, step, 0, sc.key0, sc.key1);
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    ev |= 1u << kCCand;
    if (v2 > sc.vcap2) ev |= 1u << kCOver;
    const double r = u01(u.y) * sc.nu_max;
    const double r2 = r * r;
    if (sc.kind == PIC_KIND_ELECTRON) {
        bool hit = false;
        if (r2 < R.C0 * v2) {
            double d0, d1, d2;
            iso_dir(u.z, u.w, d0, d1, d2);
            const double gg = sqrt(v2);
            vx = sc.am * vx + sc.bm * gg * d0;
            vy = sc.am * vy + sc.bm * gg * d1;
            vz = sc.am * vz + sc.bm * gg * d2;
            ev |= 1u << kCEl;
        } else if (r2 < R.C1 * v2) {
            if (v2 >= sc.v2_ex) {
                double d0, d1, d2;
                iso_dir(u.z, u.w, d0, d1, d2);
                const double gg = sqrt(v2 - sc.v2_ex);
                vx = gg * d0;
                vy = gg * d1;
                vz = gg * d2;
                ev |= 1u << kCEx;
            }
        } else if (v2 >= sc.v2_iz) {
            if (sc.rate_iz) {
                const double rr = r - R.crate;
                hit = rr < 0.0 || rr * rr < R.C1 * v2;
            } else {
                hit = r2 < R.C2 * v2;
            }
        }
        if (hit) {
            const uint4 u1 = draw(pid, step, 1, sc.key0, sc.key1);
            const double e_tot = 0.5 * v2 - sc.eps_iz;
            const double e1 = u01(u.z) * e_tot;
            const double e2 = e_tot - e1;
            const double g1 = sqrt(2.0 * e1);
            double d0, d1, d2;
            iso_dir(u1.x, u1.y, d0, d1, d2);
            vx = g1 * d0;
            vy = g1 * d1;
            vz = g1 * d2;
            iz = true;
            g2 = sqrt(2.0 * e2);
            ev |= 1u << kCIz;
        }
    } else {
        if (r2 < R.C0 * v2) {
            const uint4 u1 = draw(pid, step, 1, sc.key0, sc.key1);
            double n0, n1, n2, n3;
            box_muller(u.z, u.w, n0, n1);
            box_muller(u1.x, u1.y, n2, n3);
            vx = sc.sig_n * n0;
            vy = sc.sig_n * n1;
            vz = sc.sig_n * n2;
            ev |= 1u << kCCx;
        }
    }
}

// FP32 storage form of a position x in cells, 0 <= x < nc
__device__ __forceinline__ void split_position(double x, int nc, int32_t &cell, float &f)
{
    double c = floor(x);
    float ff = (float)(x - c);
    int32_t ci = (int32_t)c;
    if (ff >= 1.0f) {
        if (ci + 1 < nc) { ci += 1; ff = 0.0f; }
        else ff = 0x1.fffffep-1f;
    }
    cell = ci;
    f = ff;
}

}  // namespace picx
