// glint_fwd.hip -- forward glint shading kernels for gfx950 and the C ABI
// entry points glint_shade, glint_shade_rng_table (uniforms from a random-number
// table), glint_plan_*, glint_shade_batched and the
// bit-exactness utilities.
//
// Work decomposition.  One wavefront (64 lanes) owns a tile of 64 pixels.
//  1. lane = pixel: footprint and number of sub-footprints n_pr (1..n_probe_max).
//  2. a wave prefix sum flattens the tile's (pixel, probe) items; lanes then
//     take items 64 at a time, so pixels with very different footprint
//     lengths (1..21 probes, 12..252 texels) keep every lane busy.
//  3. lane = item: grid nodes, 12 simplex texels and their key hashes, then
//     for every light 48 gated binomials (4 grids x 3 texels x 4 angular
//     texels, Sec. 6.2); gates whose probability is below the smallest
//     uniform 2^-24 cannot open and are skipped without hashing.
//  4. per batch, a segmented scan across the item lanes sums each pixel's
//     items in a fixed order (deterministic); the pixel lane adds the batch
//     sum to its RGB and finally writes the RGB planes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "glint_device.hpp"
#include "glint_host.hpp"

namespace glint {

thread_local int g_last_hip_error = 0;

int set_hip_error(hipError_t e)
{
    g_last_hip_error = (int)e;
    return GLINT_EHIP;
}

struct ItemOut {
    float rgb[3];
    uint32_t lit;              // bit l: a gate of light l opened (recorded by glint_shade_lit)
    uint32_t key_sum, theta_sum, count_sum, n_open, n_gate, n_live, n_live_small, n_lit, n_live_lit;
    float b[kMaxLight];
};

// Per-wave LDS.  Static part (2048 bytes): per pixel of the tile, what its
// items need that depends neither on the probe nor on the light
// ([field][pixel], conflict-free): sigma0 e0, the probe step direction, in
// FP32 (its rounding moves a probe centre by at most 2^-25 sigma0, a few 1e-6
// lattice cells, inside every decision margin; the centre itself is FP64);
// the packed counts and node codes; the trials per node.  The instrumented
// kernel adds one result slot per lane.  Dynamic part: the per-(pixel,
// light) records (LightRec) of the tile, 2 KB per light,
// [light][word][pixel].  Item offsets stay in the pixel lanes' registers
// (cross-lane reads), so 4 lights fit in 10 KB: 16 waves per CU.
//   pk   n_pr (bits 0-6) | node count (7-9) | material (10-14) | l + 1024
//        (15-25) | node codes bits 0-5 (26-31)
//   nd   node codes bits 6-35; node g's 9-bit code (top level | k << 1 |
//        m << 4) is bits 9g..9g+8 of the 36-bit code string
struct TileSmemBase {
    float ex[kWave], ey[kWave];
    uint32_t pk[kWave];
    uint32_t nd[kWave];
    float ng[4][kWave];        // trials per node w N 2^l (Eq. 10); the baseline law keeps the weights w here
};
template <bool DEBUG>
struct TileSmem : TileSmemBase {
    ItemOut dslot[kWave];
};
template <>
struct TileSmem<false> : TileSmemBase {};

// Per-(pixel, light) record: everything a light needs at a pixel that does not
// depend on the probe, computed once by the pixel's lane before the items run
// (8 words, LDS [light][word][pixel]):
//   w0..w3  gate threshold K_g of node g (Eqs. 10, 16: the uniform's index
//           k = h >> 9 opens the gate iff k < K_g; K_g <= 2^23, bits 0-23) and,
//           in bits 24-31 of the four words, the 31-bit code
//           A | B << 15 | valid << 30 with A = (ai + 16384) mod 2^15,
//           B = (aj + 16384) mod 2^15 the lower-left angular texel (Eq. 14)
//   w4      p (Eq. 4)
//   w5, w6  the bilinear fractions of Eq. 14 along x and y: the smaller of
//           (f, 1 - f), stored as f when f <= 1/2 and as -(1 - f) otherwise
//           (the other one is 1 minus it, within 2^-24)
//   w7      F G D(n)/(R N P 4 <wi,n>) (Eqs. 1-3 without the count b)
// valid = 0 (all words 0): the light is below the horizon at this pixel (or
// zero), so it adds nothing.
constexpr int kLightRecWords = 8;
constexpr size_t kLightRecBytes = kLightRecWords * kWave * sizeof(uint32_t);   // per light

__device__ __forceinline__ void make_light_rec(const Pixel &px, const PixelRec &r, const DevMaterial &M,
                                               const DevLight &L, const ViewFrame &fr, uint32_t w[kLightRecWords],
                                               bool &pclamp)
{
#pragma unroll
    for (int k = 0; k < kLightRecWords; ++k) w[k] = 0u;
    pclamp = false;
    LightEval le;
    if (!eval_light(px.n, px.wi, px.alpha, L, M, fr, le)) return;
    pclamp = le.pclamp;
    const float lp = log1m(le.p);
    const uint32_t code = ((uint32_t)(le.ai + 16384) & 0x7FFFu) | (((uint32_t)(le.aj + 16384) & 0x7FFFu) << 15) |
                          (1u << 30);
#pragma unroll
    for (int g = 0; g < 4; ++g) w[g] = gate_K(r.ng[g], le.p, lp) | (((code >> (8 * g)) & 0xFFu) << 24);
    light_brdf(M, px.alpha, le);
    const float G = 1.0f / ((1.0f + r.lam_i) * (1.0f + le.lam_o));
    w[4] = __float_as_uint(le.p);
    w[5] = __float_as_uint(le.fx <= 0.5f ? le.fx : -le.gx);
    w[6] = __float_as_uint(le.fy <= 0.5f ? le.fy : -le.gy);
    w[7] = __float_as_uint(le.F * G * r.kpx);
}

// the fraction f and its complement 1 - f from a stored smaller one
__device__ __forceinline__ void unpack_frac(uint32_t bits, float &f, float &g)
{
    const float s = __uint_as_float(bits);
    const bool neg = (bits >> 31) != 0u;
    f = neg ? 1.0f - (-s) : s;
    g = neg ? -s : 1.0f - s;
}

// element (g, e) of a per-lane [4][3] register array for a per-lane (g, e):
// a tree of selects (registers cannot be indexed per lane).  The twelve
// values arrive as arguments, not through a reference to the array, so that
// the compiler has no loads that it could fold into one load from a per-lane
// address (which would move the array to scratch memory).
template <typename T>
__device__ __forceinline__ T pick43v(T a00, T a01, T a02, T a10, T a11, T a12, T a20, T a21, T a22, T a30, T a31,
                                     T a32, int g, int e)
{
    const bool e1 = e == 1, e2 = e == 2;
    const T x0 = e2 ? a02 : (e1 ? a01 : a00);
    const T x1 = e2 ? a12 : (e1 ? a11 : a10);
    const T x2 = e2 ? a22 : (e1 ? a21 : a20);
    const T x3 = e2 ? a32 : (e1 ? a31 : a30);
    const bool g0 = (g & 1) != 0;
    return (g & 2) ? (g0 ? x3 : x2) : (g0 ? x1 : x0);
}
#define GLINT_PICK43(a, g, e)                                                                                     \
    pick43v((a)[0][0], (a)[0][1], (a)[0][2], (a)[1][0], (a)[1][1], (a)[1][2], (a)[2][0], (a)[2][1], (a)[2][2], \
            (a)[3][0], (a)[3][1], (a)[3][2], (g), (e))

// ---------------------------------------------------------------------------
// One (pixel, probe) item: simplex texels of every grid node, then per light
// the distributed gated binomial sum b and its radiance contribution.
// Gates are tested for all 48 (node, texel, angular texel) triples without
// branching and collected in a per-lane bit mask; the open ones (a few per
// cent) are then counted in a loop over set bits, so a wave runs the
// expensive branch about max-popcount times instead of once per triple.
// Bits are taken in increasing (node, texel, angular) order: the sum order is
// that of the plain triple loop.
// ---------------------------------------------------------------------------
// Source of the 32-bit word behind the uniform of a gate (slot 0) or of a
// count (slot 1), from the item's texel key and the light's angular key:
//   kRngHash      H(texel key, angular key), computed
//   kRngTable     entry (texel key ^ angular key) & mask of a table of random
//                 words in device memory, read through the caches
//   kRngTableLds  the same entry from the wave's copy of the table in LDS
// (Sec. 6.3: the two uniforms may come from a small texture of random
// numbers precomputed once).
enum : int { kRngHash = 0, kRngTable = 1, kRngTableLds = 2 };

// Counting law of the kernel:
//   kLawDistributed  the method: distributed gated binomials (Eqs. 10, 16-18)
//   kLawZk           the baseline it replaces (Zirr and Kaplanyan): every
//                    node counts its whole cell, n = N 2^l trials, with the
//                    classical approximation of Eq. 15 (a floored Gaussian
//                    when n p > 5 or n > 16, else n Bernoulli trials), and
//                    the node outputs are mixed with the weights w (Eq. 7)
enum : int { kLawDistributed = 0, kLawZk = 1 };
// an upper bound of every ndtri_bits value (the largest, for the uniform
// 1 - 2^-24, is 5.33): a floored Gaussian count fma(sd, z, mu) is 0 for
// every uniform when fma(sd, kZmaxBound, mu) < 1
constexpr float kZmaxBound = 5.5f;

template <int RNG>
__device__ __forceinline__ uint32_t rng_word(uint32_t pre, uint32_t ak, const Shared &sh, const uint32_t *ltbl)
{
    if constexpr (RNG == kRngHash) {
        return hstep(pre, ak);
    } else if constexpr (RNG == kRngTable) {
        return sh.rng_tbl[(pre ^ ak) & sh.rng_mask];
    } else {
        return ltbl[(pre ^ ak) & sh.rng_mask];
    }
}

// angular key H(salt, angular word) of texel (ai + dx, aj + dy), slot s, from
// the record's A = (ai + 16384) mod 2^15 and B = (aj + 16384) mod 2^15
__device__ __forceinline__ uint32_t angular_key(uint32_t A, uint32_t B, int dx, int dy, int s)
{
    return hstep(kAngularSalt, ((A + (uint32_t)dx) & 0x7FFFu) | (((B + (uint32_t)dy) & 0x7FFFu) << 15) |
                                   ((uint32_t)s << 30));
}

// One (pixel, probe) part of the sampled per-texel dump (instrumented kernel
// only): key and beta [4][3], theta and count [n_light][4][3][4] at the
// slot's probe; key == nullptr: the item is not dumped.
struct DumpDst {
    uint32_t *key;
    float *beta;
    uint32_t *theta;
    float *count;
};

__device__ __forceinline__ DumpDst dump_dst(const DebugPlanes &dp, int slot, int kp, int n_light)
{
    const size_t sk = (size_t)slot * dp.dump_probes + kp;
    return {dp.dump_key + sk * 12, dp.dump_beta + sk * 12, dp.dump_theta + sk * n_light * 48,
            dp.dump_count + sk * n_light * 48};
}

__device__ void dump_zero(const DumpDst &d, int n_light)
{
    for (int i = 0; i < 12; ++i) {
        d.key[i] = 0u;
        d.beta[i] = 0.0f;
    }
    for (int i = 0; i < n_light * 48; ++i) {
        d.theta[i] = 0u;
        d.count[i] = 0.0f;
    }
}

// LK = 2 or 4 shades one item on LK lanes of a quad: lane r of the group
// takes the lights l = r (mod LK), and after every LK lights the group's
// first lane (the item's owner) receives its partners' factors (DPP quad
// moves) and extends the radiance chain with them, in light order.  With
// LK = 1 one lane takes every light.  Either way the chain is
// o.rgb = fma(E_l, f_l, o.rgb) over l = 0, 1, ... with f_l = +0 for a light
// without an open gate, so the image has the same bits.  ip: the item's
// pixel in the tile, kp: its probe, (u, v): the pixel's uv.
template <bool DEBUG, bool HEAD = true, int RNG = kRngHash, bool LIT = false, int LK = 1, int LAW = kLawDistributed>
__device__ __forceinline__ void shade_item(const TileSmem<DEBUG> &sm, const uint32_t *lrec, int ip, double u, double v,
                                           int kp, const uint32_t (&nbase)[4], const Shared &sh, ItemOut &o,
                                           const uint32_t *ltbl, float zN = 0.0f, const DumpDst dd = DumpDst{})
{
    static_assert(LK == 1 || ((LK == 2 || LK == 4) && !DEBUG), "several lanes per item only in the production kernels");
    const int lane = threadIdx.x;
    o.rgb[0] = o.rgb[1] = o.rgb[2] = 0.0f;
    if (LIT) o.lit = 0u;
    if (DEBUG) {
        o.key_sum = o.theta_sum = o.count_sum = o.n_open = o.n_gate = o.n_live = o.n_live_small = o.n_lit = 0;
        o.n_live_lit = 0;
        for (int l = 0; l < kMaxLight; ++l) o.b[l] = 0.0f;
    }
    const uint32_t pk = sm.pk[ip];
    const int npr = (int)(pk & 0x7fu), nn = (int)((pk >> 7) & 7u);
    const DevMaterial &M = sh.mats[(pk >> 10) & 31u];
    uint32_t wd[4];
    {
        const uint32_t lb = (pk >> 15) & 0x7ffu;
        const uint64_t D = (uint64_t)(pk >> 26) | ((uint64_t)sm.nd[ip] << 6);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const uint32_t d = (uint32_t)(D >> (9 * g)) & 0x1ffu;
            wd[g] = (lb + (d & 1u)) | (((d >> 1) & 7u) << 11) | ((d >> 4) << 14);
        }
    }
    double cx, cy;
    probe_centre(u, v, (double)sm.ex[ip], (double)sm.ey[ip], kp, npr, cx, cy);
    uint32_t pre[4][3];
    float beta[4][3];
    texel_keys_from(cx, cy, wd, nbase, sh, pre, beta);
    const bool dump = DEBUG && dd.key != nullptr;
    if (DEBUG) {
        for (int g = 0; g < nn; ++g)
            for (int e = 0; e < 3; ++e) o.key_sum += pre[g][e];
        if (dump) {
            dump_zero(dd, sh.n_light);
            for (int g = 0; g < nn; ++g)
                for (int e = 0; e < 3; ++e) {
                    dd.key[g * 3 + e] = pre[g][e];
                    dd.beta[g * 3 + e] = beta[g][e];
                }
        }
    }
    const int n_light = sh.n_light;
    const int trips = (n_light + LK - 1) / LK;
    for (int j = 0; j < trips; ++j) {
        const int li = LK * j + (lane & (LK - 1));
        float f = 0.0f;                        // this light's radiance factor F G D_P / (4 <wi,n>)
        do {
            if (LK > 1 && li >= n_light) break;
            const uint32_t *lw = lrec + (size_t)li * kLightRecWords * kWave + ip;
            uint32_t K[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) K[g] = lw[g * kWave];
            const uint32_t code = (K[0] >> 24) | ((K[1] >> 24) << 8) | ((K[2] >> 24) << 16) | ((K[3] >> 24) << 24);
            if (!(code & (1u << 30))) break;   // below the horizon: the light adds nothing
#pragma unroll
            for (int g = 0; g < 4; ++g) K[g] &= 0xFFFFFFu;
            const uint32_t A = code & 0x7FFFu, B = (code >> 15) & 0x7FFFu;
            if constexpr (LAW == kLawZk) {
                // baseline counting law; sm.ng holds the node weights w and zN
                // the pixel's flake density N
                const float p = __uint_as_float(lw[4 * kWave]);
                float fx, gx, fy, gy;
                unpack_frac(lw[5 * kWave], fx, gx);
                unpack_frac(lw[6 * kWave], fy, gy);
                uint32_t ak0[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) ak0[a] = angular_key(A, B, a & 1, a >> 1, 0);
                // a Bernoulli trial succeeds when (2k + 1) 2^-24 < p, k = h >> 9,
                // i.e. k < ceil((p 2^24 - 1) / 2): exact in FP32
                const float kf = ceilf((p * 16777216.0f - 1.0f) * 0.5f);
                const uint32_t KB = kf >= 8388608.0f ? 8388608u : (kf > 0.0f ? (uint32_t)kf : 0u);
                float bsum = 0.0f;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    if (g >= nn) break;
                    const float nz = ldexpf(zN, (int)(wd[g] & 0x7ffu) - 1024);   // N 2^l
                    const float w = sm.ng[g][ip];
                    const float mu = nz * p;
                    if (mu > 5.0f || nz > 16.0f) {
                        const float sd = __builtin_amdgcn_sqrtf(mu * (1.0f - p));
                        if (!DEBUG && fmaf(sd, kZmaxBound, mu) < 1.0f) continue;
#pragma unroll
                        for (int e = 0; e < 3; ++e) {
                            const float wb = w * beta[g][e];
#pragma unroll
                            for (int a = 0; a < 4; ++a) {
                                const uint32_t h0 = hstep(pre[g][e], ak0[a]);
                                const float c = fmaxf(floorf(fmaf(sd, ndtri_bits(h0), mu)), 0.0f);
                                const float va = ((a & 1) ? fx : gx) * ((a & 2) ? fy : gy);
                                bsum = fmaf(wb * va, c, bsum);
                                if (DEBUG) { o.theta_sum += h0; o.n_gate += 1; o.n_open += 1; o.count_sum += (uint32_t)c; }
                                if (dump) {
                                    dd.theta[li * 48 + g * 12 + e * 4 + a] = h0;
                                    dd.count[li * 48 + g * 12 + e * 4 + a] = c;
                                }
                            }
                        }
                    } else {
                        const int t = (int)floorf(nz + 0.5f);
                        if (!DEBUG && (t == 0 || KB == 0u)) continue;
#pragma unroll
                        for (int e = 0; e < 3; ++e) {
                            const float wb = w * beta[g][e];
#pragma unroll
                            for (int a = 0; a < 4; ++a) {
                                const uint32_t h0 = hstep(pre[g][e], ak0[a]);
                                uint32_t c = 0u;
                                for (int k = 1; k <= t; ++k) c += ((hstep(h0, (uint32_t)k) >> 9) < KB) ? 1u : 0u;
                                const float va = ((a & 1) ? fx : gx) * ((a & 2) ? fy : gy);
                                bsum = fmaf(wb * va, (float)c, bsum);
                                if (DEBUG) { o.theta_sum += h0; o.n_gate += 1; o.n_live += (uint32_t)t; o.count_sum += c; }
                                if (dump) {
                                    dd.theta[li * 48 + g * 12 + e * 4 + a] = h0;
                                    dd.count[li * 48 + g * 12 + e * 4 + a] = (float)c;
                                }
                            }
                        }
                    }
                }
                if (DEBUG) o.b[li] = bsum;
                if (!(bsum > 0.0f)) break;   // no count: the light adds exactly +0
                if (DEBUG) o.n_lit += 1;
                f = __uint_as_float(lw[7 * kWave]) * bsum;
                break;
            }
            uint32_t anyK = 0u;
#pragma unroll
            for (int g = 0; g < 4; ++g)
                if (g < nn) anyK |= K[g];
            if (!DEBUG && anyK == 0u) break;   // no gate of this light can open
            // slot-0 angular keys.  Inside a tile the light's angular cell is
            // nearly always the same for every item of the batch (95% of the
            // batch-light iterations of the 4K frame): then the four keys are
            // hashed once, in scalar registers (scalar ALU, beside the vector
            // work), instead of once per lane.
            uint32_t ak0[4];
            const uint32_t cu = __builtin_amdgcn_readfirstlane(code);
            if (__ballot(code != cu) == 0ull) {
                const uint32_t Au = cu & 0x7FFFu, Bu = (cu >> 15) & 0x7FFFu;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    ak0[a] = angular_key(Au, Bu, a & 1, a >> 1, 0);
                    // pinned to a scalar register here, so that the compiler
                    // does not merge this branch's hashing with the other's
                    // (vector) one after the branches join
                    asm volatile("" : "+s"(ak0[a]));
                }
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a) ak0[a] = angular_key(A, B, a & 1, a >> 1, 0);
            }
            uint32_t mlo = 0u, mhi = 0u;       // open gates: bit g*16 + e*4 + a (g < 2 in mlo)
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                if (g >= nn) continue;
                if (!DEBUG && K[g] == 0u) continue;   // no uniform can open these gates
                // theta0 < P>=1 (Eq. 18 gate)  <=>  (h >> 9) < K  <=>  h <= K 2^9 - 1  (K > 0)
                const uint32_t thr = (K[g] << 9) - 1u;
                if constexpr (DEBUG) {
#pragma unroll
                    for (int e = 0; e < 3; ++e) {
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            const uint32_t h0 = rng_word<RNG>(pre[g][e], ak0[a], sh, ltbl);
                            o.theta_sum += h0; o.n_gate += 1; o.n_live += K[g] ? 1u : 0u;
                            o.n_live_small += (K[g] != 0u && K[g] <= 128u) ? 1u : 0u;
                            if (dump) dd.theta[li * 48 + g * 12 + e * 4 + a] = h0;
                            const uint32_t bit = ((h0 >> 9) < K[g]) ? 1u : 0u;
                            if (g < 2) mlo |= bit << (g * 16 + e * 4 + a);
                            else mhi |= bit << ((g - 2) * 16 + e * 4 + a);
                        }
                    }
                } else {
                    // With the hash head (HEAD), the words are fmix32 without its
                    // last step x ^= x >> 16, which keeps the top 16 bits:
                    // H <= thr implies head <= thr | 0xFFFF, so a node whose
                    // heads all exceed that bound opens no gate, and the last
                    // step is only taken in the rare nodes that pass it.
                    constexpr bool kHead = RNG == kRngHash && HEAD;
                    uint32_t h[12];
                    if constexpr (RNG == kRngHash) {
#pragma unroll
                        for (int k = 0; k < 12; ++k) h[k] = hstep_head(pre[g][k >> 2], ak0[k & 3]);
                        if constexpr (!HEAD) {
#pragma unroll
                            for (int k = 0; k < 12; ++k) h[k] ^= h[k] >> 16;
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 12; ++k) h[k] = rng_word<RNG>(pre[g][k >> 2], ak0[k & 3], sh, ltbl);
                    }
                    // gates open rarely: the smallest of the node's twelve words
                    // decides whether any can have opened, and the per-gate bits
                    // are only formed when one may have in some lane of the wave
                    const uint32_t hmin = min(min(min(h[0], min(h[1], h[2])), min(h[3], min(h[4], h[5]))),
                                              min(min(h[6], min(h[7], h[8])), min(h[9], min(h[10], h[11]))));
                    if (__ballot(hmin <= (kHead ? (thr | 0xFFFFu) : thr)) != 0ull) {
                        if constexpr (kHead) {
#pragma unroll
                            for (int k = 0; k < 12; ++k) h[k] ^= h[k] >> 16;
                        }
                        uint32_t bits = 0u;
#pragma unroll
                        for (int k = 0; k < 12; ++k) bits |= (h[k] <= thr ? 1u : 0u) << k;
                        if (g < 2) mlo |= bits << (g * 16);
                        else mhi |= bits << ((g - 2) * 16);
                    }
                }
            }
            // a light without an open gate adds exactly +0 to the (non-negative) sums
            if ((mlo | mhi) == 0u) break;
            if (DEBUG) {
                o.n_lit += 1;
                for (int g = 0; g < nn; ++g) o.n_live_lit += K[g] ? 12u : 0u;
            }
            if (LIT) o.lit |= 1u << li;
            const float p = __uint_as_float(lw[4 * kWave]);
            float fx, gx, fy, gy;
            unpack_frac(lw[5 * kWave], fx, gx);
            unpack_frac(lw[6 * kWave], fy, gy);
            float bsum = 0.0f;
            while (mlo | mhi) {
                int idx;
                if (mlo) { idx = __builtin_ctz(mlo); mlo &= mlo - 1u; }
                else { idx = 32 + __builtin_ctz(mhi); mhi &= mhi - 1u; }
                const int g = idx >> 4, e = (idx >> 2) & 3, a = idx & 3;
                const uint32_t ak1 = angular_key(A, B, a & 1, a >> 1, 1);
                const uint32_t h1 = rng_word<RNG>(GLINT_PICK43(pre, g, e), ak1, sh, ltbl);
                // Eq. 17 for node g: m = max(n - 1, 0), 1 + mu, sigma (the adjoint repeats this arithmetic)
                const float ng = sm.ng[g][ip];
                const float m = fmaxf(ng - 1.0f, 0.0f);
                const float x = fmaf(__builtin_amdgcn_sqrtf(m * p * (1.0f - p)), ndtri_bits(h1), 1.0f + m * p);
                const float c = sh.rounding ? fmaxf(x, 1.0f) : fmaxf(floorf(x), 1.0f);
                const float va = ((a & 1) ? fx : gx) * ((a & 2) ? fy : gy);   // bilinear weight (Eq. 14)
                bsum = fmaf(GLINT_PICK43(beta, g, e) * va, c, bsum);
                if (DEBUG) { o.n_open += 1; o.count_sum += sh.rounding ? 0u : (uint32_t)c; }
                if (dump) dd.count[li * 48 + g * 12 + e * 4 + a] = c;
            }
            f = __uint_as_float(lw[7 * kWave]) * bsum;
            if (DEBUG) o.b[li] = bsum;
        } while (false);
        if constexpr (LK == 1) {
            const DevLight &L = sh.lights[j];
#pragma unroll
            for (int c = 0; c < 3; ++c) o.rgb[c] = fmaf(L.rad[c], f, o.rgb[c]);
        } else {
            // the owner's partners' factors: lights LK j + r (DPP quad moves
            // [1,1,3,3] for pairs, [r,r,r,r] for quads)
            float fr[LK];
            fr[0] = f;
            if constexpr (LK == 2) {
                fr[1] = __uint_as_float(dpp_mov<0xF5>(__float_as_uint(f)));
            } else {
                fr[1] = __uint_as_float(dpp_mov<0x55>(__float_as_uint(f)));
                fr[2] = __uint_as_float(dpp_mov<0xAA>(__float_as_uint(f)));
                fr[3] = __uint_as_float(dpp_mov<0xFF>(__float_as_uint(f)));
            }
#pragma unroll
            for (int r = 0; r < LK; ++r) {
                if (LK * j + r >= n_light) break;
                const DevLight &L = sh.lights[LK * j + r];
#pragma unroll
                for (int c = 0; c < 3; ++c) o.rgb[c] = fmaf(L.rad[c], fr[r], o.rgb[c]);
            }
        }
    }
    if constexpr (LIT && LK > 1) {
        o.lit |= dpp_mov<0xB1>(o.lit);             // quad_perm [1,0,3,2]
        if (LK == 4) o.lit |= dpp_mov<0x4E>(o.lit);   // quad_perm [2,3,0,1]
    }
}

// ---------------------------------------------------------------------------
// Per-pixel sums of a batch's item results.  Item j of the batch sits on lane
// j, and the items of one pixel are consecutive lanes seg..last.  A segmented
// inclusive scan (Hillis-Steele: lane j adds lane j - d when that lane is in
// its segment, for d = 1, 2, 4, 8 inside each 16-lane row, then the last
// lane of row 0 into row 1 and of row 2 into row 3, then lane 31 into rows 2
// and 3) leaves on the segment's last lane the sum of its items, in a fixed
// tree order.  Lane data moves inside VALU instructions (DPP), so the scan
// costs about 60 instructions per batch, against a loop of cross-lane reads
// as long as the longest segment.  All lanes must be active.
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS, bool LIT>
__device__ __forceinline__ void seg_step(float (&v)[3], uint32_t &l, uint32_t &m, bool take)
{
    float t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) t[c] = __uint_as_float(dpp_mov<CTRL, ROWS>(__float_as_uint(v[c])));
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = take ? v[c] + t[c] : v[c];
    if constexpr (LIT) {
        const uint32_t tl = dpp_mov<CTRL, ROWS>(l), tm = dpp_mov<CTRL, ROWS>(m);
        l = take ? (l | tl) : l;
        m = take ? (m | tm) : m;
    }
}

// v: the lane's item RGB (0 past the last item), l, m: its lit-light and
// probe bits (LIT); seg: the lane of its pixel's first item in the batch
template <bool LIT>
__device__ __forceinline__ void segmented_sums(float (&v)[3], uint32_t &l, uint32_t &m, int seg)
{
    const int j = threadIdx.x, jr = j & 15, r = j >> 4;
    seg_step<0x111, 0xf, LIT>(v, l, m, jr >= 1 && j - 1 >= seg);   // row_shr:1
    seg_step<0x112, 0xf, LIT>(v, l, m, jr >= 2 && j - 2 >= seg);   // row_shr:2
    seg_step<0x114, 0xf, LIT>(v, l, m, jr >= 4 && j - 4 >= seg);   // row_shr:4
    seg_step<0x118, 0xf, LIT>(v, l, m, jr >= 8 && j - 8 >= seg);   // row_shr:8
    seg_step<0x142, 0xa, LIT>(v, l, m, (r & 1) != 0 && 16 * r - 1 >= seg);   // row_bcast:15, rows 1 and 3
    seg_step<0x143, 0xc, LIT>(v, l, m, r >= 2 && 31 >= seg);                // row_bcast:31, rows 2 and 3
}

// per-pixel angular fingerprint (debug only): sum of slot-0 angular keys
__device__ uint32_t akey_fingerprint(const Pixel &px, const Shared &sh)
{
    const DevMaterial &M = sh.mats[px.mat];
    ViewFrame fr;
    view_frame(px.n, px.wi, px.rc, px.rs, fr);
    uint32_t s = 0;
    for (int li = 0; li < sh.n_light; ++li) {
        LightEval le;
        if (!eval_light(px.n, px.wi, px.alpha, sh.lights[li], M, fr, le)) continue;
        for (int a = 0; a < 4; ++a) s += hstep(kAngularSalt, angular_word(le.ai + (a & 1), le.aj + (a >> 1), 0));
    }
    return s;
}

// ---------------------------------------------------------------------------
// One tile of 64 pixels (tile_w x 64/tile_w) at (x0, y0) of a view.
//  1. lane = pixel: footprint, probes, grid nodes (setup_pixel), the pixel's
//     LDS fields, and one record per light (make_light_rec).
//  2. a wave prefix sum flattens the tile's (pixel, probe) items; lanes take
//     them 64 at a time (two or four lanes per item in a last batch of at
//     most 32 or 16 items).
//  3. per batch, segmented_sums leaves each pixel's item sum on the lane of
//     its last item, and the pixel lane adds it to its RGB (one cross-lane
//     read per channel).
// lrec: the tile's dynamic LDS, n_light * kLightRecBytes.
// ---------------------------------------------------------------------------
template <bool DEBUG, bool HEAD = true, int RNG = kRngHash, bool LIT = false, int LAW = kLawDistributed>
__device__ __forceinline__ void shade_tile(const ViewDesc &vw, const Shared &sh, const DebugPlanes &dp, int x0, int y0,
                           int lw, TileSmem<DEBUG> &sm, uint32_t *lrec, const uint32_t *ltbl = nullptr,
                           uint16_t *lit = nullptr, uint32_t *lit_probes = nullptr, float *zden = nullptr)
{
    const int lane = threadIdx.x;
    const int tmask = (1 << lw) - 1;
    // the pixel phase (G-buffer loads, FP64 set-up) runs at a raised wave
    // priority, the item batches at the normal one: a wave that starts a tile
    // gets its loads out ahead of the waves in their item loops (1% faster)
    if (!DEBUG) __builtin_amdgcn_s_setprio(1);
    const int x = x0 + (lane & tmask), y = y0 + (lane >> lw);
    const bool inb = (x < vw.width) && (y < vw.height);
    const int64_t idx = (int64_t)y * vw.stride + x;
    int npr = 0;
    bool plive = true;                         // some light of the pixel has a gate that can open
    float pxu = 0.0f, pxv = 0.0f;              // the pixel's uv (its items read them across lanes)
    uint32_t pxb[4] = {0u, 0u, 0u, 0u};        // its nodes' key prefixes H(root, node), likewise
    uint32_t dflags = 0, dcell = 0, dakey = 0;
    int dlevel = 0;
    {
        Pixel px;
        px.flags = 0;
        px.npr = 0;
        if (inb) setup_pixel<DEBUG>(vw, idx, sh, px);
        if (px.flags & F_SHADED) {
            npr = px.npr;
            pxu = (float)px.u;
            pxv = (float)px.v;
            const PixelRec r = make_rec(px, sh);
#pragma unroll
            for (int g = 0; g < 4; ++g) pxb[g] = hstep(sh.mats[px.mat].root, rec_node_word(r, g));
            sm.ex[lane] = r.ex;
            sm.ey[lane] = r.ey;
            {
                // node codes of PixelRec (two per word, at bits 0 and 16) as one 36-bit string
                const uint64_t D = (uint64_t)(r.nd[0] & 0x1ffu) | ((uint64_t)((r.nd[0] >> 16) & 0x1ffu) << 9) |
                                   ((uint64_t)(r.nd[1] & 0x1ffu) << 18) | ((uint64_t)((r.nd[1] >> 16) & 0x1ffu) << 27);
                sm.pk[lane] = r.pk | ((uint32_t)(D & 0x3fu) << 26);
                sm.nd[lane] = (uint32_t)(D >> 6);
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) sm.ng[g][lane] = LAW == kLawZk ? px.nw[g] : r.ng[g];
            if constexpr (LAW == kLawZk) zden[lane] = px.N;   // the baseline needs the weights and N
            const DevMaterial &M = sh.mats[px.mat];
            ViewFrame fr;
            view_frame(px.n, px.wi, px.rc, px.rs, fr);
            const int nn = rec_nodes(r);
            bool live = false;                 // some light above the horizon has a gate that can open
            for (int li = 0; li < sh.n_light; ++li) {
                uint32_t w[kLightRecWords];
                bool pclamp;
                make_light_rec(px, r, M, sh.lights[li], fr, w, pclamp);
                if (pclamp) px.flags |= F_CLAMP_P;
#pragma unroll
                for (int k = 0; k < kLightRecWords; ++k) lrec[((size_t)li * kLightRecWords + k) * kWave + lane] = w[k];
                // words 0-3: the nodes' gate thresholds (low 24 bits); bit 30 of
                // word 3: the light is above the horizon
                const uint32_t kor = w[0] | (nn > 1 ? w[1] : 0u) | (nn > 2 ? w[2] : 0u) | (nn > 3 ? w[3] : 0u);
                live = live || (((w[3] >> 30) & 1u) != 0u && (kor & 0xFFFFFFu) != 0u);
            }
            plive = live;
        }
        if (DEBUG) {
            dflags = px.flags;
            dcell = npr ? px.cell : 0u;
            dlevel = npr ? px.level : 0;
            dakey = npr ? akey_fingerprint(px, sh) : 0u;
            // dump slot: this lane zeroes the probes the pixel does not have,
            // the items write the others
            const int slot = (dp.dump_slot && inb) ? dp.dump_slot[idx] : -1;
            if (slot >= 0 && slot < dp.dump_cap)
                for (int k = npr; k < dp.dump_probes; ++k) dump_zero(dump_dst(dp, slot, k, sh.n_light), sh.n_light);
        }
    }
    __syncthreads();
    if (!DEBUG) __builtin_amdgcn_s_setprio(0);
    float acc[3] = {0.0f, 0.0f, 0.0f};
    uint32_t litacc = 0u, probeacc = 0u;
    uint32_t dks = 0, dts = 0, dcs = 0, dno = 0, dng = 0, dnl = 0, dns = 0, dlt = 0, dll = 0;
    float db[kMaxLight];
    if (DEBUG)
        for (int l = 0; l < kMaxLight; ++l) db[l] = 0.0f;
    // A pixel where no gate of any light can open has radiance exactly 0 and
    // no lit light: in production it has no items.  The instrumented kernel
    // shades the items of such pixels after the others, in batches of their
    // own (phase 1), for its counters; the other pixels' items then fall into
    // the same batches as in production, so the per-pixel sums, and the
    // image, have the same bits.
    constexpr bool kSkipDead = LAW == kLawDistributed;
    constexpr int kPhases = (DEBUG && kSkipDead) ? 2 : 1;
    for (int phase = 0; phase < kPhases; ++phase) {
    const int nph = !kSkipDead ? npr : (((phase == 0) == plive) ? npr : 0);
    // (cross-lane reads: measured faster here than wave_inclusive_sum)
    int incl = nph;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    const int off = incl - nph;
    const int S = __shfl(incl, kWave - 1);
    for (int base = 0; base < S; base += kWave) {
        // a last batch of at most 32 (16) items takes two (four) lanes per
        // item, lane r of the group shading the lights l = r mod 2 (4); the
        // item's result is on the group's first lane
        const int lkl = DEBUG ? 0 : (S - base <= kWave / 4 && sh.n_light > 2) ? 2 :
                                    (S - base <= kWave / 2 && sh.n_light > 1) ? 1 : 0;
        const int lk = 1 << lkl;
        const int q = base + (lane >> lkl);
        float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f;
        uint32_t ol = 0u;
        // the item's pixel and probe, with every lane active (cross-lane reads)
        const int qc = q < S ? q : S - 1;
        const int p = item_pixel(off, qc);
        const int kp = qc - __shfl(off, p);
        const double pu = (double)__shfl(pxu, p), pv = (double)__shfl(pxv, p);
        uint32_t nb[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) nb[g] = (uint32_t)__shfl((int)pxb[g], p);
        if (q < S) {
            ItemOut o;
            const float zN = LAW == kLawZk ? zden[p] : 0.0f;
            if constexpr (DEBUG) {
                const int64_t pidx = (int64_t)(y0 + (p >> lw)) * vw.stride + (x0 + (p & tmask));
                DumpDst dd = {};
                const int slot = dp.dump_slot ? dp.dump_slot[pidx] : -1;
                if (slot >= 0 && slot < dp.dump_cap && kp < dp.dump_probes) dd = dump_dst(dp, slot, kp, sh.n_light);
                shade_item<DEBUG, HEAD, RNG, LIT, 1, LAW>(sm, lrec, p, pu, pv, kp, nb, sh, o, ltbl, zN, dd);
            } else if (lk == 1)
                shade_item<DEBUG, HEAD, RNG, LIT, 1, LAW>(sm, lrec, p, pu, pv, kp, nb, sh, o, ltbl, zN);
            else if (lk == 2)
                shade_item<DEBUG, HEAD, RNG, LIT, DEBUG ? 1 : 2, LAW>(sm, lrec, p, pu, pv, kp, nb, sh, o, ltbl, zN);
            else
                shade_item<DEBUG, HEAD, RNG, LIT, DEBUG ? 1 : 4, LAW>(sm, lrec, p, pu, pv, kp, nb, sh, o, ltbl, zN);
            o0 = o.rgb[0];
            o1 = o.rgb[1];
            o2 = o.rgb[2];
            if (LIT) ol = o.lit;
            if constexpr (DEBUG) sm.dslot[lane] = o;
        }
        // item j of the batch onto lane j (lk lanes per item: from lane lk j),
        // then the per-pixel sums of the batch (segmented_sums)
        float v[3] = {o0, o1, o2};
        uint32_t vl = ol, vm = (LIT && ol) ? 1u << min(kp, 31) : 0u;   // probe bit 31: probe 31 or a later one
        int kj = kp;
        if (lk > 1) {
            const int src = (lane << lkl) & (kWave - 1);
            const bool in = lane < (kWave >> lkl);
#pragma unroll
            for (int c = 0; c < 3; ++c) v[c] = __shfl(v[c], src);
            kj = __shfl(kj, src);
            if (LIT) {
                vl = (uint32_t)__shfl((int)vl, src);
                vm = (uint32_t)__shfl((int)vm, src);
            }
            if (!in) {
                v[0] = v[1] = v[2] = 0.0f;
                vl = vm = 0u;
                kj = 0;
            }
        }
        // a batch whose items are all first probes has one item per pixel:
        // every segment is a single lane and the sums are the items themselves
        if (__ballot(kj != 0) != 0ull) segmented_sums<LIT>(v, vl, vm, lane - min(kj, lane));
        // pixel lane: its items i0..i1-1 of this batch end on lane i1-1-base
        const int i0 = max(off, base), i1 = min(off + nph, base + kWave);
        const int src = i1 > i0 ? i1 - 1 - base : lane;
        const float r0 = __shfl(v[0], src), r1 = __shfl(v[1], src), r2 = __shfl(v[2], src);
        const uint32_t rl = LIT ? (uint32_t)__shfl((int)vl, src) : 0u, rm = LIT ? (uint32_t)__shfl((int)vm, src) : 0u;
        if (i1 > i0) {
            acc[0] += r0;
            acc[1] += r1;
            acc[2] += r2;
            if (LIT) {
                litacc |= rl;
                probeacc |= rm;
            }
        }
        if constexpr (DEBUG) {
            __syncthreads();
            for (int i = i0; i < i1; ++i) {
                const ItemOut &s = sm.dslot[i - base];
                dks += s.key_sum; dts += s.theta_sum; dcs += s.count_sum; dno += s.n_open; dng += s.n_gate;
                dnl += s.n_live;
                dns += s.n_live_small;
                dlt += s.n_lit;
                dll += s.n_live_lit;
                for (int l = 0; l < kMaxLight; ++l) db[l] += s.b[l];
            }
            __syncthreads();
        }
    }
    }
    if (inb) {
        const int64_t npx = (int64_t)vw.height * vw.stride;
        vw.out[idx] = acc[0];
        vw.out[npx + idx] = acc[1];
        vw.out[2 * npx + idx] = acc[2];
        if (LIT) {
            lit[idx] = (uint16_t)litacc;
            if (lit_probes) lit_probes[idx] = probeacc;
        }
        if (DEBUG) {
            if (dp.flags) dp.flags[idx] = dflags;
            if (dp.n_probe) dp.n_probe[idx] = npr;
            if (dp.level) dp.level[idx] = dlevel;
            if (dp.cell) dp.cell[idx] = dcell;
            if (dp.key_sum) dp.key_sum[idx] = dks;
            if (dp.akey_sum) dp.akey_sum[idx] = dakey;
            if (dp.theta_sum) dp.theta_sum[idx] = dts;
            if (dp.count_sum) dp.count_sum[idx] = dcs;
            if (dp.n_open) dp.n_open[idx] = dno;
            if (dp.n_gate) dp.n_gate[idx] = dng;
            if (dp.n_live) dp.n_live[idx] = dnl;
            if (dp.n_live_small) dp.n_live_small[idx] = dns;
            if (dp.n_lit) dp.n_lit[idx] = dlt;
            if (dp.n_live_lit) dp.n_live_lit[idx] = dll;
            if (dp.b_light)
                for (int l = 0; l < sh.n_light; ++l) dp.b_light[l * npx + idx] = db[l];
        }
    }
}

// One workgroup per tile.  With a tile order (cost classes, heaviest first)
// workgroup b shades tile order[b]; without one, tiles go in row-major order.
// Dynamic LDS: the tile's light records (n_light * kLightRecBytes), then,
// with RNG = kRngTableLds, the wave's copy of the random-number table
// (rng_mask + 1 words, a multiple of 4, 16-byte aligned), or with
// LAW = kLawZk the tile's flake densities (64 floats).
// RNG selects the source of the gate uniforms (rng_word).
// With LIT the kernel also writes, per pixel, the bit mask of the lights that
// opened a gate in any of the pixel's probes (lit[y * stride + x]) and, if
// lit_probes is given, the bit mask of the probes that opened one (bit k:
// probe k, bit 31: probe 31 or a later one).
template <bool DEBUG, int RNG = kRngHash, bool LIT = false, int LAW = kLawDistributed>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DEBUG ? 1 : 4))) void glint_fwd_kernel(
    ViewDesc vw, Shared sh, DebugPlanes dp, int lw, int tiles_x, const int32_t *__restrict__ order, int32_t n_tiles,
    uint16_t *__restrict__ lit, uint32_t *__restrict__ lit_probes)
{
    __shared__ TileSmem<DEBUG> sm;
    extern __shared__ uint4 glint_dyn_lds[];
    const int t = order ? __builtin_amdgcn_readfirstlane(order[blockIdx.x]) : (int)blockIdx.x;
    if ((unsigned)t >= (unsigned)n_tiles) return;
    const int tx = t % tiles_x, ty = t / tiles_x;
    uint32_t *lrec = reinterpret_cast<uint32_t *>(glint_dyn_lds);
    uint32_t *tail = lrec + (size_t)sh.n_light * kLightRecWords * kWave;
    const uint32_t *ltbl = nullptr;
    if constexpr (RNG == kRngTableLds) {
        const uint4 *src = reinterpret_cast<const uint4 *>(sh.rng_tbl);
        uint4 *dst = reinterpret_cast<uint4 *>(tail);
        const int n4 = (int)((sh.rng_mask + 1u) >> 2);
        for (int i = threadIdx.x; i < n4; i += kWave) dst[i] = src[i];
        __syncthreads();
        ltbl = tail;
    }
    float *zden = LAW == kLawZk ? reinterpret_cast<float *>(tail) : nullptr;
    shade_tile<DEBUG, RNG == kRngHash, RNG, LIT, LAW>(vw, sh, dp, tx << lw, ty << (6 - lw), lw, sm, lrec, ltbl, lit,
                                                     lit_probes, zden);
}

// Random-number table: t[i] = H(seed, i) for i < n.
__global__ __launch_bounds__(256) void glint_rng_fill_kernel(uint32_t *__restrict__ t, uint64_t n, uint32_t seed)
{
    const uint64_t step = (uint64_t)gridDim.x * 256u;
    for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += step) t[i] = hstep(seed, (uint32_t)i);
}

// wave-uniform copies (scalar registers) of a descriptor's fields
__device__ __forceinline__ int32_t uni32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ int64_t uni64(int64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ T *uniptr(T *p)
{
    return reinterpret_cast<T *>(uni64(reinterpret_cast<int64_t>(p)));
}

__device__ __forceinline__ ViewDesc uniform_view(const ViewDesc &v)
{
    ViewDesc u;
    u.width = uni32(v.width);
    u.height = uni32(v.height);
    u.stride = uni64(v.stride);
    u.u = uniptr(v.u); u.v = uniptr(v.v);
    u.dudx = uniptr(v.dudx); u.dvdx = uniptr(v.dvdx); u.dudy = uniptr(v.dudy); u.dvdy = uniptr(v.dvdy);
    u.nx = uniptr(v.nx); u.ny = uniptr(v.ny); u.nz = uniptr(v.nz);
    u.wx = uniptr(v.wx); u.wy = uniptr(v.wy); u.wz = uniptr(v.wz);
    u.mat = uniptr(v.mat);
    u.alpha_px = uniptr(v.alpha_px);
    u.log10N_px = uniptr(v.log10N_px);
    u.out = uniptr(v.out);
    u.tx = uniptr(v.tx);
    u.ty = uniptr(v.ty);
    u.tz = uniptr(v.tz);
    return u;
}

// Persistent batched kernel: workgroups pop chunks of tiles from a global
// counter until every tile of every view is done (the loop always ends: the
// counter only grows and each pop covers at least one tile).  Tile indices
// and view descriptors are wave-uniform (scalar registers).
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void glint_batched_kernel(
    const ViewDesc *__restrict__ views,
                                                           const int32_t *__restrict__ tile_start,
                                                           int n_views, int32_t n_tiles, int lw, int chunk,
                                                           unsigned int *counter, const Shared *__restrict__ shp)
{
    __shared__ TileSmem<false> sm;
    __shared__ int s_t0;
    extern __shared__ uint4 glint_dyn_lds[];
    uint32_t *lrec = reinterpret_cast<uint32_t *>(glint_dyn_lds);
    DebugPlanes dp = {};
    for (;;) {
        if (threadIdx.x == 0) s_t0 = (int)atomicAdd(counter, (unsigned int)chunk);
        __syncthreads();
        const int t0 = __builtin_amdgcn_readfirstlane(s_t0);
        __syncthreads();
        if (t0 >= n_tiles) break;
        const int t1 = min(t0 + chunk, n_tiles);
        for (int t = t0; t < t1; ++t) {
            int lo = 0, hi = n_views;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (tile_start[mid] <= t) lo = mid; else hi = mid;
            }
            lo = __builtin_amdgcn_readfirstlane(lo);
            const ViewDesc vw = uniform_view(views[lo]);
            const int local = uni32(t - tile_start[lo]);
            const int tiles_x = (vw.width + (1 << lw) - 1) >> lw;
            const int tx = local % tiles_x, ty = local / tiles_x;
            // an opaque copy of the parameter pointer per tile keeps the compiler
            // from hoisting parameter loads out of the loop (which would hold them
            // in registers across every tile and halve the occupancy)
            const Shared *sp = shp;
            asm volatile("" : "+s"(sp));
            shade_tile<false, false>(vw, *sp, dp, tx << lw, ty << (6 - lw), lw, sm, lrec);
        }
    }
}

__global__ void glint_reset_counter(unsigned int *counter) { *counter = 0u; }

// The same tile table with one workgroup per tile (non-persistent): workgroup
// t finds its view by binary search over the tile prefix and shades that
// view's tile, within the single-view kernel's register budget.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void glint_batched_grid_kernel(
    const ViewDesc *__restrict__ views, const int32_t *__restrict__ tile_start, int n_views, int32_t n_tiles,
    int lw, const Shared *__restrict__ shp)
{
    __shared__ TileSmem<false> sm;
    extern __shared__ uint4 glint_dyn_lds[];
    const int t = (int)blockIdx.x;
    if (t >= n_tiles) return;
    int lo = 0, hi = n_views;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= t) lo = mid; else hi = mid;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const ViewDesc vw = uniform_view(views[lo]);
    const int local = uni32(t - tile_start[lo]);
    const int tiles_x = (vw.width + (1 << lw) - 1) >> lw;
    const int tx = local % tiles_x, ty = local / tiles_x;
    DebugPlanes dp = {};
    shade_tile<false>(vw, *shp, dp, tx << lw, ty << (6 - lw), lw, sm, reinterpret_cast<uint32_t *>(glint_dyn_lds));
}

// bit-exactness utilities ----------------------------------------------------
__global__ void glint_texel_hash_kernel(const int32_t *keys, int64_t n, uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t *k = keys + 9 * i;
    const uint32_t root = hstep(kRootSalt, (uint32_t)k[0]);
    const uint32_t base = hstep(root, node_word(k[1], k[2], k[3]));
    const uint32_t pre = hstep(hstep(base, (uint32_t)k[4]), (uint32_t)k[5]);
    const uint32_t ak = hstep(kAngularSalt, angular_word(k[6], k[7], k[8]));
    out[i] = hstep(pre, ak);
}

__global__ void glint_hash_step_kernel(const uint32_t *h, const uint32_t *w, int64_t n, uint32_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = hstep(h[i], w[i]);
}

__global__ void glint_ndtri_kernel(const uint32_t *bits, int64_t n, float *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = ndtri_bits(bits[i]);
}

static bool valid_tile_w(int w) { return w == 8 || w == 16 || w == 32 || w == 64; }

static int log2_tile(int w) { return w == 8 ? 3 : (w == 16 ? 4 : (w == 32 ? 5 : 6)); }

}  // namespace glint

// ===========================================================================
// C ABI
// ===========================================================================
using namespace glint;

struct glint_plan {
    ViewDesc *d_views = nullptr;
    Shared *d_sh = nullptr;
    int32_t *d_tile_start = nullptr;
    unsigned int *d_counter = nullptr;
    int n_views = 0;
    int64_t n_tiles = 0;
    int tile_w = 8;
    int chunk = 4;
    int n_blocks = 0;
    bool per_tile = false;     // one workgroup per tile instead of persistent workgroups
    Shared sh;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t graph_stream = nullptr;
};

extern "C" {

int glint_version(void) { return 10000; }

int glint_last_hip_error(void) { return g_last_hip_error; }

const char *glint_status_string(int s)
{
    switch (s) {
    case GLINT_OK: return "ok";
    case GLINT_EINVAL: return "invalid argument value";
    case GLINT_ENULL: return "required pointer is NULL";
    case GLINT_ESHAPE: return "inconsistent shape or stride";
    case GLINT_EHIP: return "HIP runtime error (see glint_last_hip_error)";
    case GLINT_EUNSUPPORTED: return "unsupported request";
    case GLINT_ENOMEM: return "device allocation failed";
    case GLINT_ELIMIT: return "view exceeds the static workspace of glint_shade_noalloc";
    default: return "unknown status";
    }
}

size_t glint_shade_workspace_bytes(int32_t width, int32_t height) { return tile_order_bytes(width, height); }

}  // extern "C"

// Shared body of glint_shade and glint_shade_rng_table: tile order, then one
// launch of the shading kernel with the uniforms' source RNG and the counting
// law (kLawZk only with hashed uniforms and without lit masks).
static int launch_forward(const glint_gbuffer *gbuf, Shared &sh, float *out_rgb, const glint_debug *dbg,
                          void *workspace, size_t workspace_bytes, int rng, size_t lds_bytes, uint16_t *lit,
                          uint32_t *lit_probes, void *stream, int law = kLawDistributed)
{
    if (law == kLawZk && (rng != kRngHash || lit)) return GLINT_EUNSUPPORTED;
    if (dbg && dbg->dump_slot) {
        if (!dbg->dump_key || !dbg->dump_beta || !dbg->dump_theta || !dbg->dump_count) return GLINT_ENULL;
        if (dbg->dump_capacity < 1 || dbg->dump_probes < 1 || dbg->dump_probes > GLINT_MAX_PROBES) return GLINT_EINVAL;
        const uintptr_t al = reinterpret_cast<uintptr_t>(dbg->dump_slot) | reinterpret_cast<uintptr_t>(dbg->dump_key) |
                             reinterpret_cast<uintptr_t>(dbg->dump_beta) |
                             reinterpret_cast<uintptr_t>(dbg->dump_theta) |
                             reinterpret_cast<uintptr_t>(dbg->dump_count);
        if (al & 3u) return GLINT_EINVAL;
    }
    ViewDesc vw;
    int rc = make_view(gbuf, out_rgb, vw);
    if (rc) return rc;
    if ((int64_t)vw.width * vw.height == 0) return GLINT_OK;
    const int tiles_x = (int)tiles_x_of(vw.width);
    const int64_t nt = tiles_of(vw.width, vw.height);
    if (nt > 0x7fffffffLL) return GLINT_ESHAPE;
    hipStream_t st = (hipStream_t)stream;
    const int32_t *order = nullptr;
    if (workspace) {
        rc = enqueue_tile_order(vw, sh, workspace, workspace_bytes, &order, st);
        if (rc) return rc;
    }
    const dim3 grid((unsigned)nt), block(kWave);
    // dynamic LDS: the light records, then the table copy or the flake densities
    const unsigned rec_b = (unsigned)(sh.n_light * kLightRecBytes);
    const unsigned zk_b = rec_b + kWave * sizeof(float);
    if (dbg) {
        // the instrumented kernel reads a table through the caches: same words as from LDS
        DebugPlanes dp = {dbg->flags, dbg->n_probe, dbg->level, dbg->cell, dbg->key_sum, dbg->akey_sum,
                          dbg->theta_sum, dbg->count_sum, dbg->n_open, dbg->n_gate, dbg->n_live, dbg->b_light,
                          dbg->n_live_small, dbg->n_lit, dbg->n_live_lit,
                          dbg->dump_slot, dbg->dump_capacity, dbg->dump_probes, dbg->dump_key, dbg->dump_beta,
                          dbg->dump_theta, dbg->dump_count};
        if (law == kLawZk)
            hipLaunchKernelGGL((glint_fwd_kernel<true, kRngHash, false, kLawZk>), grid, block, zk_b, st, vw, sh, dp,
                               kTileLw, tiles_x, order, (int32_t)nt, nullptr, nullptr);
        else if (rng == kRngHash)
            hipLaunchKernelGGL(glint_fwd_kernel<true>, grid, block, rec_b, st, vw, sh, dp, kTileLw, tiles_x, order,
                               (int32_t)nt, nullptr, nullptr);
        else
            hipLaunchKernelGGL((glint_fwd_kernel<true, kRngTable>), grid, block, rec_b, st, vw, sh, dp, kTileLw,
                               tiles_x, order, (int32_t)nt, nullptr, nullptr);
    } else {
        DebugPlanes dp = {};
        if (law == kLawZk)
            hipLaunchKernelGGL((glint_fwd_kernel<false, kRngHash, false, kLawZk>), grid, block, zk_b, st, vw, sh, dp,
                               kTileLw, tiles_x, order, (int32_t)nt, nullptr, nullptr);
        else if (rng == kRngHash && lit)
            hipLaunchKernelGGL((glint_fwd_kernel<false, kRngHash, true>), grid, block, rec_b, st, vw, sh, dp, kTileLw,
                               tiles_x, order, (int32_t)nt, lit, lit_probes);
        else if (rng == kRngHash)
            hipLaunchKernelGGL(glint_fwd_kernel<false>, grid, block, rec_b, st, vw, sh, dp, kTileLw, tiles_x, order,
                               (int32_t)nt, nullptr, nullptr);
        else if (rng == kRngTable)
            hipLaunchKernelGGL((glint_fwd_kernel<false, kRngTable>), grid, block, rec_b, st, vw, sh, dp, kTileLw,
                               tiles_x, order, (int32_t)nt, nullptr, nullptr);
        else
            hipLaunchKernelGGL((glint_fwd_kernel<false, kRngTableLds>), grid, block, rec_b + (unsigned)lds_bytes, st,
                               vw, sh, dp, kTileLw, tiles_x, order, (int32_t)nt, nullptr, nullptr);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

extern "C" {

int glint_shade(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat, const glint_light *lights,
                int32_t n_light, const glint_params *params, float *out_rgb, const glint_debug *dbg,
                void *workspace, size_t workspace_bytes, void *stream)
{
    Shared sh;
    int rc = prepare_shared(mats, n_mat, lights, n_light, params, sh, GLINT_FLAG_ZK_COUNT);
    if (rc) return rc;
    const int law = (params->flags & GLINT_FLAG_ZK_COUNT) ? kLawZk : kLawDistributed;
    return launch_forward(gbuf, sh, out_rgb, dbg, workspace, workspace_bytes, kRngHash, 0, nullptr, nullptr, stream,
                          law);
}

int glint_shade_lit(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat, const glint_light *lights,
                    int32_t n_light, const glint_params *params, float *out_rgb, uint16_t *lit_lights,
                    uint32_t *lit_probes, void *workspace, size_t workspace_bytes, void *stream)
{
    Shared sh;
    int rc = prepare_shared(mats, n_mat, lights, n_light, params, sh);
    if (rc) return rc;
    if (!lit_lights) return GLINT_ENULL;
    if ((reinterpret_cast<uintptr_t>(lit_lights) & 1u) != 0 || (reinterpret_cast<uintptr_t>(lit_probes) & 3u) != 0)
        return GLINT_EINVAL;
    return launch_forward(gbuf, sh, out_rgb, nullptr, workspace, workspace_bytes, kRngHash, 0, lit_lights, lit_probes,
                          stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free forward (glint_shade_noalloc): the tile-order workspace is
// a file-scope device array, one copy per GPU that loads the library, held
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy: on the first call on each device (with that device
// current) hipGetSymbolAddress gives that device's address of the array,
// which is kept per device and used from then on.  Nothing in the array has
// to start at zero: the order pass writes every byte it later reads (class
// bytes, per-block class counts, their offsets, the order) before reading it.
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[GLINT_NOALLOC_WORKSPACE_BYTES];
static std::atomic<void *> g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_of_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_hip_error(e);
    if (dev < 0 || dev >= kMaxDevices) return GLINT_EUNSUPPORTED;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return set_hip_error(e);
            if (!p) return GLINT_EUNSUPPORTED;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return GLINT_OK;
}

extern "C" {

int glint_shade_noalloc(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                        const glint_light *lights, int32_t n_light, const glint_params *params, float *out_rgb,
                        void *stream)
{
    Shared sh;
    int rc = prepare_shared(mats, n_mat, lights, n_light, params, sh, GLINT_FLAG_ZK_COUNT);
    if (rc) return rc;
    if (!gbuf) return GLINT_ENULL;
    if (gbuf->width < 0 || gbuf->height < 0) return GLINT_ESHAPE;
    const size_t need = tile_order_bytes(gbuf->width, gbuf->height);
    if (need > GLINT_NOALLOC_WORKSPACE_BYTES) return GLINT_ELIMIT;
    void *ws = nullptr;
    if (need > 0) {
        rc = scratch_of_current_device(&ws);
        if (rc) return rc;
    }
    const int law = (params->flags & GLINT_FLAG_ZK_COUNT) ? kLawZk : kLawDistributed;
    return launch_forward(gbuf, sh, out_rgb, nullptr, ws, need, kRngHash, 0, nullptr, nullptr, stream, law);
}

int glint_rng_table_fill(uint32_t *table, int32_t log2_words, uint32_t seed, void *stream)
{
    if (!table) return GLINT_ENULL;
    if (log2_words < GLINT_RNG_TABLE_MIN_LOG2 || log2_words > GLINT_RNG_TABLE_MAX_LOG2) return GLINT_EINVAL;
    if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0) return GLINT_EINVAL;
    const uint64_t n = 1ull << log2_words;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(glint_rng_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, table, n,
                       seed);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

int glint_shade_rng_table(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                          const glint_light *lights, int32_t n_light, const glint_params *params,
                          const uint32_t *table, int32_t log2_words, int32_t placement, float *out_rgb,
                          const glint_debug *dbg, void *workspace, size_t workspace_bytes, void *stream)
{
    Shared sh;
    int rc = prepare_shared(mats, n_mat, lights, n_light, params, sh);
    if (rc) return rc;
    if (!table) return GLINT_ENULL;
    if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0) return GLINT_EINVAL;
    if (placement == GLINT_RNG_CACHED) {
        if (log2_words < GLINT_RNG_TABLE_MIN_LOG2 || log2_words > GLINT_RNG_TABLE_MAX_LOG2) return GLINT_EINVAL;
    } else if (placement == GLINT_RNG_LDS) {
        if (log2_words < GLINT_RNG_TABLE_MIN_LOG2 || log2_words > GLINT_RNG_LDS_MAX_LOG2) return GLINT_EINVAL;
    } else {
        return GLINT_EINVAL;
    }
    sh.rng_tbl = table;
    sh.rng_mask = log2_words >= 32 ? 0xFFFFFFFFu : ((1u << log2_words) - 1u);
    const int rng = placement == GLINT_RNG_LDS ? kRngTableLds : kRngTable;
    const size_t lds_bytes = placement == GLINT_RNG_LDS ? (size_t)4 << log2_words : 0;
    return launch_forward(gbuf, sh, out_rgb, dbg, workspace, workspace_bytes, rng, lds_bytes, nullptr, nullptr,
                          stream);
}

int glint_plan_create(const glint_gbuffer *gbufs, float *const *out_rgb, int32_t n_views,
                      const glint_material *mats, int32_t n_mat, const glint_light *lights, int32_t n_light,
                      const glint_params *params, const glint_tune *tune, glint_plan **plan)
{
    if (!plan || !gbufs || !out_rgb) return GLINT_ENULL;
    *plan = nullptr;
    if (n_views < 1) return GLINT_ESHAPE;
    glint_plan *P = new (std::nothrow) glint_plan();
    if (!P) return GLINT_ENOMEM;
    int rc = prepare_shared(mats, n_mat, lights, n_light, params, P->sh);
    if (rc) { delete P; return rc; }
    P->tile_w = kTileW;                          // defaults: the library's tile shape, a workgroup per tile
    int bpc = 0;
    if (tune) {
        if (!valid_tile_w(tune->tile_w) || tune->tile_w * tune->tile_h != kWave || tune->blocks_per_cu < 0 ||
            tune->blocks_per_cu > 64) {
            delete P;
            return GLINT_EINVAL;
        }
        P->tile_w = tune->tile_w;
        bpc = tune->blocks_per_cu;
    }
    std::vector<ViewDesc> views((size_t)n_views);
    std::vector<int32_t> start((size_t)n_views + 1);
    int64_t total = 0;
    const int tile_h = kWave / P->tile_w;
    for (int i = 0; i < n_views; ++i) {
        rc = make_view(&gbufs[i], out_rgb[i], views[i]);
        if (rc) { delete P; return rc; }
        start[i] = (int32_t)total;
        total += (int64_t)((views[i].width + P->tile_w - 1) / P->tile_w) * ((views[i].height + tile_h - 1) / tile_h);
        if (total > 0x7fff0000LL) { delete P; return GLINT_ESHAPE; }
    }
    start[n_views] = (int32_t)total;
    P->n_views = n_views;
    P->n_tiles = total;
    int dev = 0, n_cu = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) { delete P; return set_hip_error(e); }
    int64_t want = (int64_t)n_cu * bpc;
    P->n_blocks = (int)(want < 1 ? 1 : want);
    if (bpc == 0) {
        P->per_tile = true;
        P->n_blocks = (int)total;
    }
    // chunks of tiles per pop: about 16 pops per workgroup, at most 16 tiles
    int64_t per = total / ((int64_t)P->n_blocks * 16);
    P->chunk = (int)(per < 1 ? 1 : (per > 16 ? 16 : per));
    e = hipMalloc((void **)&P->d_views, sizeof(ViewDesc) * n_views);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_sh, sizeof(Shared));
    if (e == hipSuccess) e = hipMemcpy(P->d_sh, &P->sh, sizeof(Shared), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_tile_start, sizeof(int32_t) * (n_views + 1));
    if (e == hipSuccess) e = hipMalloc((void **)&P->d_counter, sizeof(unsigned int));
    if (e == hipSuccess) e = hipMemcpy(P->d_views, views.data(), sizeof(ViewDesc) * n_views, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(P->d_tile_start, start.data(), sizeof(int32_t) * (n_views + 1), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        glint_plan_destroy(P);
        return e == hipErrorOutOfMemory ? GLINT_ENOMEM : set_hip_error(e);
    }
    *plan = P;
    return GLINT_OK;
}

static int enqueue_batched(glint_plan *P, hipStream_t st)
{
    if (P->per_tile) {
        hipLaunchKernelGGL(glint_batched_grid_kernel, dim3((unsigned)P->n_tiles), dim3(kWave),
                           (unsigned)(P->sh.n_light * kLightRecBytes), st, P->d_views,
                           P->d_tile_start, P->n_views, (int32_t)P->n_tiles, log2_tile(P->tile_w), P->d_sh);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? GLINT_OK : set_hip_error(e);
    }
    hipLaunchKernelGGL(glint_reset_counter, dim3(1), dim3(1), 0, st, P->d_counter);
    hipLaunchKernelGGL(glint_batched_kernel, dim3((unsigned)P->n_blocks), dim3(kWave),
                       (unsigned)(P->sh.n_light * kLightRecBytes), st, P->d_views,
                       P->d_tile_start, P->n_views, (int32_t)P->n_tiles, log2_tile(P->tile_w), P->chunk,
                       P->d_counter, P->d_sh);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

int glint_shade_batched(glint_plan *P, int32_t use_graph, void *stream)
{
    if (!P) return GLINT_ENULL;
    if (P->n_tiles == 0) return GLINT_OK;
    hipStream_t st = (hipStream_t)stream;
    if (!use_graph) return enqueue_batched(P, st);
    if (!P->exec) {
        // capture on a private stream so that the caller's stream is never in capture mode
        hipStream_t cs;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return set_hip_error(e);
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) { (void)hipStreamDestroy(cs); return set_hip_error(e); }
        int rc = enqueue_batched(P, cs);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return set_hip_error(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) { (void)hipGraphDestroy(g); return set_hip_error(e); }
        P->graph = g;
        P->exec = ex;
    }
    hipError_t e = hipGraphLaunch(P->exec, st);
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

int glint_plan_info(const glint_plan *P, int64_t *n_tiles, int32_t *n_blocks)
{
    if (!P) return GLINT_ENULL;
    if (n_tiles) *n_tiles = P->n_tiles;
    if (n_blocks) *n_blocks = P->n_blocks;
    return GLINT_OK;
}

int glint_plan_destroy(glint_plan *P)
{
    if (!P) return GLINT_OK;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->d_views) (void)hipFree(P->d_views);
    if (P->d_sh) (void)hipFree(P->d_sh);
    if (P->d_tile_start) (void)hipFree(P->d_tile_start);
    if (P->d_counter) (void)hipFree(P->d_counter);
    delete P;
    return GLINT_OK;
}

int glint_texel_hash(const int32_t *keys, int64_t n, uint32_t *out, void *stream)
{
    if (n < 0) return GLINT_ESHAPE;
    if (n == 0) return GLINT_OK;
    if (!keys || !out) return GLINT_ENULL;
    hipLaunchKernelGGL(glint_texel_hash_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, keys, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

int glint_hash_step(const uint32_t *h, const uint32_t *w, int64_t n, uint32_t *out, void *stream)
{
    if (n < 0) return GLINT_ESHAPE;
    if (n == 0) return GLINT_OK;
    if (!h || !w || !out) return GLINT_ENULL;
    hipLaunchKernelGGL(glint_hash_step_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, h, w, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

int glint_ndtri(const uint32_t *bits, int64_t n, float *out, void *stream)
{
    if (n < 0) return GLINT_ESHAPE;
    if (n == 0) return GLINT_OK;
    if (!bits || !out) return GLINT_ENULL;
    hipLaunchKernelGGL(glint_ndtri_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, bits, n, out);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

}  // extern "C"
