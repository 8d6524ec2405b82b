// glint_bwd.hip -- adjoint of the relaxed glint forward for gfx950 and the C
// ABI entry points glint_backward_workspace_bytes / glint_shade_backward.
//
// The adjoint recomputes the forward at the current parameters, so every
// discrete decision (probe split, area level, ratio/orientation cell,
// triangle, tetrahedron, lattice triangle, angular cell, gate, the max(1,x)
// clamp and the p <= 1 clamp) is exactly the forward's; only the continuous
// part of the relaxed count c = max(1, 1 + mu + sigma z) is differentiated
// (straight-through floor).  Parameters: each material's roughness alpha
// and log flake density ln N, each light's raw direction.
//
// Reduction (deterministic): per light, a fixed-order wave sum by DPP lane
// moves (wave_sum); per material, fixed-order LDS sums in the tile kernel and
// wave sums in the work-unit kernel; per tile or work unit, one
// partial row in the workspace (row index = tile index, so the sums do not
// depend on the order in which tiles run); two FP64 kernels then sum the rows
// in a fixed order.  Tiles run heaviest first (the forward's tile order).
//
// Every gradient term of a light is proportional to its distributed count b,
// which is zero unless one of its gates opened.  Given the forward's record
// of which lights opened a gate in each pixel (glint_shade_lit), the adjoint
// shades only the pixels with one, gathered into full waves, and in those
// only the lights with one: the same terms, without recomputing the gates
// that the forward found closed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "glint_device.hpp"
#include "glint_host.hpp"

namespace glint {

// v + (v moved across lanes by the DPP control CTRL, dpp_mov)
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_add(float v)
{
    return v + __uint_as_float(dpp_mov<CTRL, ROWS>(__float_as_uint(v)));
}

// Sum over the 64 lanes (every lane active), in a fixed order, with data
// moves between lanes inside the VALU instructions (no LDS round trips):
// pairs, quads, 8 and 16 lanes of a row, then row 0 into row 1 and row 2
// into row 3, then rows 0-1 into row 3; lane 63 holds the total, which is
// returned to every lane.
__device__ __forceinline__ float wave_sum(float v)
{
    v = dpp_add<0xB1>(v);          // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E>(v);          // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141>(v);         // row_half_mirror
    v = dpp_add<0x140>(v);         // row_mirror
    v = dpp_add<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Per-wave LDS (10176 bytes: 16 workgroups per CU).  As in the forward,
// column `lane` of pre[][] is private to the lane while its item runs;
// afterwards rows 0-2 hold the item's (material, d/d alpha, d/d ln N) for the
// fixed-order per-material sums.
struct BwdSmem {
    int off[kWave];
    PixelRec rec[kWave];
    uint32_t pre[12][kWave];
    float beta[12][kWave];
    float dd[kMaxLight][3];
};

// The adjoint terms of one light at one (pixel, probe) item: adds d/d alpha
// and d/d ln N of the item's material to da, dn and returns d/d dir of the
// light in gd.  Returns whether one of the light's gates opened: otherwise
// every term is exactly zero (each is proportional to a distributed count or
// to one of its derivatives).  Gates are collected in bit masks and the open
// ones processed in a compacted loop, as in the forward.
__device__ __forceinline__ bool light_grad(const PixelRec &R, const double n[3], const double wi[3],
                                           const DevMaterial &M, const ViewFrame &fr, const uint32_t (&pre)[4][3],
                                           int nn, float alpha, float kpx, float lam_i, float dli_da, float inv_micro,
                                           const DevLight &L, const float gout[3], BwdSmem &sm, float &da, float &dn,
                                           float gd[3])
{
    const int lane = threadIdx.x;
    gd[0] = gd[1] = gd[2] = 0.0f;
    LightEval le;
    if (!eval_light(n, wi, alpha, L, M, fr, le)) return false;
    const float s = gout[0] * L.rad[0] + gout[1] * L.rad[1] + gout[2] * L.rad[2];
    const float p = le.p;
    const float lp = log1m(p);
    uint32_t K[4], anyK = 0u;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        K[g] = gate_K(R.ng[g], p, lp);
        if (g < nn) anyK |= K[g];
    }
    uint32_t mlo = 0u, mhi = 0u;
    if (anyK) {
        uint32_t ak0[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            ak0[a] = hstep(kAngularSalt, angular_word(le.ai + (a & 1), le.aj + (a >> 1), 0));
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g >= nn || K[g] == 0u) continue;
            const uint32_t thr = (K[g] << 9) - 1u;   // (h >> 9) < K  <=>  h <= K 2^9 - 1
#pragma unroll
            for (int e = 0; e < 3; ++e) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const uint32_t bit = (hstep(pre[g][e], ak0[a]) <= thr) ? 1u : 0u;
                    if (g < 2) mlo |= bit << (g * 16 + e * 4 + a);
                    else mhi |= bit << ((g - 2) * 16 + e * 4 + a);
                }
            }
        }
    }
    float B = 0.0f, Bp = 0.0f, Bm = 0.0f, Bfx = 0.0f, Bfy = 0.0f;
    const bool opened = (mlo | mhi) != 0u;
    while (mlo | mhi) {
        int idx;
        if (mlo) { idx = __builtin_ctz(mlo); mlo &= mlo - 1u; }
        else { idx = 32 + __builtin_ctz(mhi); mhi &= mhi - 1u; }
        const int g = idx >> 4, e = (idx >> 2) & 3, a = idx & 3;
        const int ge = g * 3 + e;
        const uint32_t ak1 = hstep(kAngularSalt, angular_word(le.ai + (a & 1), le.aj + (a >> 1), 1));
        const uint32_t h1 = hstep(sm.pre[ge][lane], ak1);
        const float z = ndtri_bits(h1);
        // Eq. 17 for node g (same arithmetic as the forward)
        const float ng = R.ng[g];
        const float m = fmaxf(ng - 1.0f, 0.0f);
        const float sgg = __builtin_amdgcn_sqrtf(m * p * (1.0f - p));
        const float x = fmaf(sgg, z, 1.0f + m * p);
        const float be = sm.beta[ge][lane];
        const float wx = (a & 1) ? le.fx : le.gx, wy = (a & 2) ? le.fy : le.gy;
        const float va = wx * wy;                             // bilinear weight (Eq. 14)
        const float dvx = (a & 1) ? wy : -wy, dvy = (a & 2) ? wx : -wx;
        if (x >= 1.0f) {                                      // relaxed count c = x
            const float isg = sgg > 0.0f ? 0.5f / sgg : 0.0f;
            const float dsdp = m * (1.0f - 2.0f * p) * isg;   // d sigma / d p
            const float dsdm = p * (1.0f - p) * isg;          // d sigma / d m
            const float dmdl = ng > 1.0f ? ng : 0.0f;         // d m / d ln N
            const float bv = be * va;
            B = fmaf(bv, x, B);
            Bp = fmaf(bv, m + z * dsdp, Bp);
            Bm = fmaf(bv, (p + z * dsdm) * dmdl, Bm);
            Bfx = fmaf(be * dvx, x, Bfx);
            Bfy = fmaf(be * dvy, x, Bfy);
        } else {                                              // clamped: c = 1
            B = fmaf(be, va, B);
            Bfx += be * dvx;
            Bfy += be * dvy;
        }
    }
    // Every term below is proportional to one of B, Bp, Bm, Bfx, Bfy, which
    // are exactly 0 without an open gate: such lanes skip the algebra.
    if (!opened) return false;
    light_brdf(M, alpha, le);
    // derivatives of p (Eq. 4) with respect to alpha and c2 = <n,h>^2
    const float c2 = (float)(le.ch * le.ch), s2 = (float)(1.0 - le.ch * le.ch);
    const float a2 = alpha * alpha;
    float dp_da = 0.0f, dp_dc2 = 0.0f;
    if (!le.pclamp && p > 0.0f) {
        if (M.ndf == 0) {
            const float d = s2 + c2 * a2;
            dp_da = 4.0f * p / alpha * (1.0f - a2 * c2 / d);
            dp_dc2 = 2.0f * p * (1.0f - a2) / d;
        } else {
            dp_da = 2.0f * p * s2 / (c2 * a2 * alpha);
            dp_dc2 = p * (1.0f / (c2 * c2 * a2) - 2.0f / c2);
        }
    }
    const float co = (float)le.cos_o, so2 = (float)(1.0 - le.cos_o * le.cos_o);
    float dlo_dc, dlo_da;
    smith_lambda_grad(M.ndf, alpha, co, so2, dlo_dc, dlo_da);
    const float G = 1.0f / ((1.0f + lam_i) * (1.0f + le.lam_o));
    const float dG_da = -G * (dli_da / (1.0f + lam_i) + dlo_da / (1.0f + le.lam_o));
    const float sk = s * kpx;
    da += sk * (le.F * dG_da * B + le.F * G * Bp * dp_da) - 2.0f * sk * le.F * G * B / alpha;
    dn += sk * le.F * G * (Bm - B);
    // gradient with respect to the unit half vector h
    // the unit half vector itself (the forward needs only its dot products)
    const double h[3] = {(wi[0] + L.wo[0]) * le.ihl, (wi[1] + L.wo[1]) * le.ihl, (wi[2] + L.wo[2]) * le.ihl};
    const float om = (float)(1.0 - (wi[0] * h[0] + wi[1] * h[1] + wi[2] * h[2]));
    const float dF = -5.0f * (1.0f - M.F0) * om * om * om * om * G * B;   // times wi
    const float cn = sk * le.F * G * Bp * dp_dc2 * 2.0f * (float)le.ch;   // times n
    const float ct = sk * le.F * G * Bfx * inv_micro;                      // times t
    const float cb = sk * le.F * G * Bfy * inv_micro;                      // times b
    double ta[3], ba[3];
    frame_axes(n, fr, ta, ba);
    float gh[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        gh[c] = sk * dF * (float)wi[c] + cn * (float)n[c] + ct * (float)ta[c] + cb * (float)ba[c];
    // direct dependence on wo through Lambda(<n,wo>)
    const float gon = sk * le.F * B * (-G / (1.0f + le.lam_o)) * dlo_dc;
    // h = (wi + wo)/|wi + wo|, wo = d/|d|: chain through both normalisations
    const float hx = (float)h[0], hy = (float)h[1], hz = (float)h[2];
    const float hd = gh[0] * hx + gh[1] * hy + gh[2] * hz;
    const float ihl = (float)le.ihl;
    const float gw[3] = {(gh[0] - hd * hx) * ihl + gon * (float)n[0],
                         (gh[1] - hd * hy) * ihl + gon * (float)n[1],
                         (gh[2] - hd * hz) * ihl + gon * (float)n[2]};
    const float wxl = (float)L.wo[0], wyl = (float)L.wo[1], wzl = (float)L.wo[2];
    const float wd = gw[0] * wxl + gw[1] * wyl + gw[2] * wzl;
    const float idl = L.inv_len;
    gd[0] = (gw[0] - wd * wxl) * idl;
    gd[1] = (gw[1] - wd * wyl) * idl;
    gd[2] = (gw[2] - wd * wzl) * idl;
    return true;
}

// one (pixel, probe) item: accumulates d/d alpha and d/d ln N of the pixel's
// material into da, dn, and d/d dir of each light into sm.dd (wave-reduced).
// Called by every lane of the wave (live = false contributes zeros).
// Lights whose bit in litm is clear are skipped: the forward opened none of
// their gates in this pixel, so they contribute exactly zero.
__device__ void grad_item(bool live, const PixelRec &R, double u, double v, const double n[3], const double wi[3],
                          double rc, double rs, int kp, const Shared &sh, const float gout[3], uint32_t litm,
                          float &da, float &dn, BwdSmem &sm)
{
    da = 0.0f;
    dn = 0.0f;
    const int lane = threadIdx.x;
    const int nn = live ? rec_nodes(R) : 0;
    const DevMaterial &M = sh.mats[live ? rec_mat(R) : 0];
    uint32_t pre[4][3];
    if (live) probe_texels(R, u, v, kp, M, sh, pre, sm, (uint32_t *)nullptr);
    ViewFrame fr = {};
    if (live) view_frame(n, wi, rc, rs, fr);
    const float alpha = live ? R.alpha : 1.0f;
    const float kpx = live ? R.kpx : 0.0f, lam_i = live ? R.lam_i : 0.0f;
    float dli_da = 0.0f, dl_dc;                 // d Lambda(view) / d alpha
    if (live)
        smith_lambda_grad(M.ndf, alpha, (float)fr.cos_i, (float)(1.0 - fr.cos_i * fr.cos_i), dl_dc, dli_da);
    const float inv_micro = (float)M.inv_micro;
    for (int li = 0; li < sh.n_light; ++li) {
        const DevLight &L = sh.lights[li];
        float gd[3];
        bool opened = false;                     // this lane opened a gate of this light
        if (live && ((litm >> li) & 1u))
            opened = light_grad(R, n, wi, M, fr, pre, nn, alpha, kpx, lam_i, dli_da, inv_micro, L, gout, sm, da, dn, gd);
        else
            gd[0] = gd[1] = gd[2] = 0.0f;
        float gdx = gd[0], gdy = gd[1], gdz = gd[2];
        if (__ballot(opened) != 0ull) {          // uniform: every lane takes part in the sums
            gdx = wave_sum(gdx);
            gdy = wave_sum(gdy);
            gdz = wave_sum(gdz);
            if (lane == 0) {
                sm.dd[li][0] += gdx;
                sm.dd[li][1] += gdy;
                sm.dd[li][2] += gdz;
            }
        }
    }
}

// one (pixel, probe, light) item of the masked adjoint, light li being the
// lane's own: d/d alpha and d/d ln N of the pixel's material (da, dn) and
// d/d dir of light li (gd).  Lanes with live = false return zeros.
__device__ __forceinline__ void grad_item_light(bool live, const PixelRec &R, double u, double v, const double n[3],
                                const double wi[3], double rc, double rs, int kp, int li, const Shared &sh,
                                const float gout[3], float &da, float &dn, float gd[3], BwdSmem &sm)
{
    da = 0.0f;
    dn = 0.0f;
    gd[0] = gd[1] = gd[2] = 0.0f;
    if (!live) return;
    const int nn = rec_nodes(R);
    const DevMaterial &M = sh.mats[rec_mat(R)];
    uint32_t pre[4][3];
    probe_texels(R, u, v, kp, M, sh, pre, sm, (uint32_t *)nullptr);
    ViewFrame fr;
    view_frame(n, wi, rc, rs, fr);
    float dli_da, dl_dc;                          // d Lambda(view) / d alpha
    smith_lambda_grad(M.ndf, R.alpha, (float)fr.cos_i, (float)(1.0 - fr.cos_i * fr.cos_i), dl_dc, dli_da);
    light_grad(R, n, wi, M, fr, pre, nn, R.alpha, R.kpx, R.lam_i, dli_da, (float)M.inv_micro, sh.lights[li], gout,
               sm, da, dn, gd);
}

// Work units: without a lit mask, workgroup b shades the tile order[b]
// (heaviest first); with one, workgroup b takes the lit pixels
// list[64 b .. 64 b + 63] (raster order, built by the compaction passes
// below), so that the few lit pixels fill whole waves.  The partial row is
// that of the tile, or of the chunk b.
// lit (nullable): the forward's per-pixel mask of lights with an open gate;
// only the lights of a pixel whose bit is set are evaluated.  lit_probes
// (nullable): the forward's per-pixel mask of probes with an open gate (bit
// 31: probe 31 or a later one); only those probes become items.

// position of the j-th set bit (from 0) of m, which has more than j set bits
__device__ __forceinline__ int nth_bit(uint32_t m, int j)
{
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const int c = __popc(m & ((1u << w) - 1u));
        if (j >= c) {
            j -= c;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void glint_bwd_kernel(
    ViewDesc vw, Shared sh, const float *gout, const uint16_t *__restrict__ lit,
    const uint32_t *__restrict__ lit_probes, const uint32_t *__restrict__ list, const uint32_t *__restrict__ list_len,
    int tiles_x, const int32_t *__restrict__ order, int32_t n_tiles, float *partials, int n_par, int row_stride)
{
    __shared__ BwdSmem sm;
    const int lane = threadIdx.x;
    constexpr int tile_w = kTileW, tile_h = kTileH;
    int row;
    bool inb;
    int64_t idx;
    if (list) {
        const uint32_t len = __builtin_amdgcn_readfirstlane(list_len[0]);
        const uint32_t q = blockIdx.x * (uint32_t)kWave + (uint32_t)lane;
        if (blockIdx.x * (uint32_t)kWave >= len) return;
        row = (int)blockIdx.x;
        inb = q < len;
        idx = inb ? (int64_t)list[q] : 0;
    } else {
        const int tile = order ? __builtin_amdgcn_readfirstlane(order[blockIdx.x]) : (int)blockIdx.x;
        if ((unsigned)tile >= (unsigned)n_tiles) return;
        row = tile;
        const int x0 = (tile % tiles_x) * tile_w, y0 = (tile / tiles_x) * tile_h;
        const int x = x0 + (lane % tile_w), y = y0 + (lane / tile_w);
        inb = (x < vw.width) && (y < vw.height);
        idx = (int64_t)y * vw.stride + x;
    }
    const int64_t npx = (int64_t)vw.height * vw.stride;
    int npr = 0;                               // items of this pixel
    uint32_t pmask = 0xffffffffu;              // its probes that become items (all ones: every probe)
    {
        Pixel px;
        px.flags = 0;
        px.npr = 0;
        if (inb && (!lit || lit[idx] != 0)) setup_pixel<false>(vw, idx, sh, px);
        if (px.flags & F_SHADED) {
            npr = px.npr;
            sm.rec[lane] = make_rec(px, sh);
            if (lit_probes && npr <= 31) {
                pmask = lit_probes[idx] & ((1u << npr) - 1u);
                npr = __popc(pmask);
            }
        }
    }
    const int incl = wave_inclusive_sum(npr);
    const int S = __builtin_amdgcn_readlane(incl, kWave - 1);
    sm.off[lane] = incl - npr;
    if (lane < kMaxLight * 3) (&sm.dd[0][0])[lane] = 0.0f;
    __syncthreads();
    float acc_a = 0.0f, acc_n = 0.0f;          // lane m < n_mat: material m
    for (int base = 0; base < S; base += kWave) {
        const int q = base + lane;
        const bool live = q < S;
        int p = 0, kp = 0;
#pragma unroll
        for (int st = 32; st > 0; st >>= 1)
            if (sm.off[p + st] <= q) p += st;
        const int64_t pidx = __shfl(idx, p);     // the item's pixel (all lanes take part)
        const uint32_t pm = __shfl(pmask, p);
        float g3[3] = {0.0f, 0.0f, 0.0f};
        uint32_t litm = 0u;
        double n[3] = {0, 0, 1}, wi[3] = {0, 0, 1}, u = 0.0, v = 0.0, rc = 1.0, rs = 0.0;
        if (live) {
            kp = q - sm.off[p];
            if (pm != 0xffffffffu) kp = nth_bit(pm, kp);
            normalize_in(vw.nx[pidx], vw.ny[pidx], vw.nz[pidx], n);
            normalize_in(vw.wx[pidx], vw.wy[pidx], vw.wz[pidx], wi);
            if (vw.tx) tangent_rotation(n, vw.tx[pidx], vw.ty[pidx], vw.tz[pidx], rc, rs);
            u = vw.u[pidx];
            v = vw.v[pidx];
            g3[0] = gout[pidx];
            g3[1] = gout[npx + pidx];
            g3[2] = gout[2 * npx + pidx];
            litm = lit ? (uint32_t)lit[pidx] : 0xffffffffu;
        }
        float da, dn;
        grad_item(live, sm.rec[p], u, v, n, wi, rc, rs, kp, sh, g3, litm, da, dn, sm);
        sm.pre[0][lane] = live ? (uint32_t)rec_mat(sm.rec[p]) : 0xffffffffu;
        sm.pre[1][lane] = __float_as_uint(da);
        sm.pre[2][lane] = __float_as_uint(dn);
        __syncthreads();
        if (lane < sh.n_mat) {
            for (int j = 0; j < kWave; ++j) {
                if (sm.pre[0][j] == (uint32_t)lane) {
                    acc_a += __uint_as_float(sm.pre[1][j]);
                    acc_n += __uint_as_float(sm.pre[2][j]);
                }
            }
        }
        __syncthreads();
    }
    // row of this tile: [alpha, lnN] per material, then 3 per light, zero padding to row_stride
    float *prow = partials + (int64_t)row * row_stride;
    for (int c0 = 0; c0 < row_stride; c0 += kWave) {       // uniform loop: every lane takes part in the shuffles
        const int c = c0 + lane;
        const int m = (c >> 1) & (kWave - 1);                // material of column c (lane m holds its sums)
        const float va = __shfl(acc_a, m), vn = __shfl(acc_n, m);
        float v = 0.0f;
        if (c < 2 * sh.n_mat) v = (c & 1) ? vn : va;
        else if (c < n_par) v = (&sm.dd[0][0])[c - 2 * sh.n_mat];
        if (c < row_stride) prow[c] = v;
    }
}

// ---------------------------------------------------------------------------
// Masked adjoint in balanced work units.  With both masks the items are
// (pixel, lit probe, lit light) triples, so each lane evaluates one light and
// no lane waits on a light another lane needs.  Chunk c is the lit-list
// entries [64c, 64c + 64); its items are numbered pixel by pixel (probe
// rank major, light rank minor) and cut into batches of 64, the work units.
// A fixed grid of kUnitGroups workgroups (four per wave slot of the chip, so
// that slots freed early take further ranges) takes contiguous ranges of
// units (the same number each), redoes a chunk's pixel set-up only when its
// range enters that chunk, and writes one partial row per workgroup: the
// sums run in a fixed order whatever the schedule.
// ---------------------------------------------------------------------------
constexpr int kUnitWaves = 4;          // chunks per workgroup of the count pass
constexpr int kUnitGroups = 16384;     // workgroups (partial rows) of the unit kernel: four per wave slot

// probe items of a lit pixel: its probes with an open gate (bit k: probe k;
// bit 31: probes 31 to npr - 1)
__device__ __forceinline__ int lit_probe_count(uint32_t pm, int npr)
{
    return __popc(pm & 0x7fffffffu) + ((pm >> 31) ? max(npr - 31, 0) : 0);
}

// nb[c] = number of 64-item batches of chunk c, for the chunks of the list
// (a grid-stride loop over them)
__global__ __launch_bounds__(kWave * kUnitWaves) void glint_unit_count(ViewDesc vw, Shared sh,
                                                                         const uint16_t *__restrict__ lit,
                                                                         const uint32_t *__restrict__ lit_probes,
                                                                         const uint32_t *__restrict__ list,
                                                                         const uint32_t *__restrict__ list_len,
                                                                         int64_t n_chunks, uint32_t *__restrict__ nb)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t len = list_len[0];
    const int64_t used = (len + kWave - 1) / kWave < n_chunks ? (len + kWave - 1) / kWave : n_chunks;
    const uint32_t lmask = (1u << sh.n_light) - 1u;
    const int64_t waves = (int64_t)gridDim.x * kUnitWaves;
    for (int64_t c = (int64_t)blockIdx.x * kUnitWaves + (int)(threadIdx.x / kWave); c < used; c += waves) {
        const int64_t e = c * kWave + lane;
        int cnt = 0;
        if (e < len) {
            const uint32_t idx = list[e];
            const uint32_t pm = lit_probes[idx];
            int npr = 0;
            if (pm >> 31) {                    // probes from 31 on: the pixel's probe count
                Pixel px;
                px.flags = 0;
                px.npr = 0;
                setup_pixel<false>(vw, idx, sh, px);
                npr = px.npr;
            }
            cnt = lit_probe_count(pm, npr) * __popc((uint32_t)lit[idx] & lmask);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (lane == 0) nb[c] = (uint32_t)((cnt + kWave - 1) / kWave);
    }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void glint_bwd_unit_kernel(
    ViewDesc vw, Shared sh, const float *gout, const uint16_t *__restrict__ lit,
    const uint32_t *__restrict__ lit_probes, const uint32_t *__restrict__ list, const uint32_t *__restrict__ list_len,
    const uint32_t *__restrict__ unit_off, const uint32_t *__restrict__ n_units_p, float *partials, int n_par,
    int row_stride)
{
    __shared__ BwdSmem sm;
    const int lane = threadIdx.x;
    const int64_t npx = (int64_t)vw.height * vw.stride;
    const uint32_t lmask = (1u << sh.n_light) - 1u;
    const uint32_t len = (uint32_t)__builtin_amdgcn_readfirstlane((int)list_len[0]);
    const uint32_t n_units = (uint32_t)__builtin_amdgcn_readfirstlane((int)n_units_p[0]);
    const uint32_t n_chunks = (len + kWave - 1) / kWave;
    const uint32_t per = (n_units + gridDim.x - 1) / gridDim.x;
    uint32_t u = blockIdx.x * per;
    const uint32_t u_end = min(u + per, n_units);
    if (lane < kMaxLight * 3) (&sm.dd[0][0])[lane] = 0.0f;
    __syncthreads();
    float acc_a = 0.0f, acc_n = 0.0f;          // lane m < n_mat: material m
    if (u < u_end) {
        // the chunk of unit u: the last c with unit_off[c] <= u (every chunk of
        // the list has at least one batch, and unit_off[0] = 0), by 64-way search
        uint32_t lo = 0, hi = n_chunks;
        while (hi - lo > 1) {
            const uint32_t step = (hi - lo + kWave - 1) / kWave;
            const uint32_t pos = lo + (uint32_t)lane * step;
            const uint64_t m = __ballot(pos < hi && unit_off[pos] <= u);
            lo += (uint32_t)(63 - __clzll(m)) * step;
            hi = min(lo + step, hi);
        }
        uint32_t c = lo;
        uint32_t b = u - (uint32_t)__builtin_amdgcn_readfirstlane((int)unit_off[c]);
        int cur = -1, S = 0;
        // the chunk lane's pixel: its first item, list entry and masks
        int offr = 0;
        uint32_t pixr = 0u, pmr = 0u, litr = 0u;
        while (u < u_end && c < n_chunks) {
            if ((int)c != cur) {
                // the chunk's pixel set-up: records (probe count 0 for a pixel
                // that is not shaded) and the first item of each pixel
                __syncthreads();               // the previous chunk's records are no longer read
                const uint32_t e = c * kWave + (uint32_t)lane;
                const bool has = e < len;
                const uint32_t pix = has ? list[e] : 0u;
                const uint32_t pm = has ? lit_probes[pix] : 0u;
                const uint32_t litm = has ? ((uint32_t)lit[pix] & lmask) : 0u;
                Pixel px;
                px.flags = 0;
                px.npr = 0;
                if (has) setup_pixel<false>(vw, pix, sh, px);
                if (px.flags & F_SHADED) sm.rec[lane] = make_rec(px, sh);
                else sm.rec[lane].pk = 0u;
                const int cnt = has ? lit_probe_count(pm, px.npr) * __popc(litm) : 0;
                const int incl = wave_inclusive_sum(cnt);
                S = __builtin_amdgcn_readlane(incl, kWave - 1);
                offr = incl - cnt;
                pixr = pix;
                pmr = pm;
                litr = litm;
                cur = (int)c;
                __syncthreads();
            }
            if (S == 0) {                      // no item (masks that disagree): no unit either
                ++c;
                b = 0;
                continue;
            }
            // batch b of chunk c: item r -> pixel p (the last with off <= r),
            // then probe rank r' / nl and light rank r' % nl, r' = r - off
            const int r = (int)b * kWave + lane;
            // cross-lane reads from the chunk lanes, every lane active
            const int p = item_pixel(offr, r < S ? r : S - 1);
            const int offp = __shfl(offr, p);
            const uint32_t pidx = (uint32_t)__shfl((int)pixr, p), pm = (uint32_t)__shfl((int)pmr, p);
            const uint32_t litm = (uint32_t)__shfl((int)litr, p);
            const bool live = r < S && rec_npr(sm.rec[p]) > 0;
            int kp = 0, li = 0;
            float g3[3] = {0.0f, 0.0f, 0.0f};
            double n[3] = {0, 0, 1}, wi[3] = {0, 0, 1}, uu = 0.0, vv = 0.0, rc = 1.0, rs = 0.0;
            if (live) {
                const int nl = __popc(litm);
                const int rr = r - offp;
                const int pr = rr / nl, lr = rr - pr * nl;
                const uint32_t low = pm & 0x7fffffffu;
                const int nlow = __popc(low);
                kp = pr < nlow ? nth_bit(low, pr) : 31 + (pr - nlow);
                li = nth_bit(litm, lr);
                normalize_in(vw.nx[pidx], vw.ny[pidx], vw.nz[pidx], n);
                normalize_in(vw.wx[pidx], vw.wy[pidx], vw.wz[pidx], wi);
                if (vw.tx) tangent_rotation(n, vw.tx[pidx], vw.ty[pidx], vw.tz[pidx], rc, rs);
                uu = vw.u[pidx];
                vv = vw.v[pidx];
                g3[0] = gout[pidx];
                g3[1] = gout[npx + pidx];
                g3[2] = gout[2 * npx + pidx];
            }
            float da, dn, gd[3];
            grad_item_light(live, sm.rec[p], uu, vv, n, wi, rc, rs, kp, li, sh, g3, da, dn, gd, sm);
            // per material and per light, a wave sum over the lanes of that
            // material or light (fixed order); lane m keeps material m's sums
            const int mat = live ? rec_mat(sm.rec[p]) : -1;
            for (int m = 0; m < sh.n_mat; ++m) {
                const bool mine = mat == m;
                if (__ballot(mine) == 0ull) continue;
                const float xa = wave_sum(mine ? da : 0.0f);
                const float xn = wave_sum(mine ? dn : 0.0f);
                if (lane == m) {
                    acc_a += xa;
                    acc_n += xn;
                }
            }
            for (int l = 0; l < sh.n_light; ++l) {
                const bool mine = live && li == l;
                if (__ballot(mine) == 0ull) continue;
                const float x = wave_sum(mine ? gd[0] : 0.0f);
                const float y = wave_sum(mine ? gd[1] : 0.0f);
                const float z = wave_sum(mine ? gd[2] : 0.0f);
                if (lane == 0) {
                    sm.dd[l][0] += x;
                    sm.dd[l][1] += y;
                    sm.dd[l][2] += z;
                }
            }
            __syncthreads();                   // this item's texel columns are free again
            ++u;
            if ((int)(++b) * kWave >= S) {
                ++c;
                b = 0;
            }
        }
    }
    // this workgroup's row: [alpha, lnN] per material, then 3 per light, zero padding
    float *prow = partials + (int64_t)blockIdx.x * row_stride;
    for (int c0 = 0; c0 < row_stride; c0 += kWave) {
        const int col = c0 + lane;
        const int m = (col >> 1) & (kWave - 1);
        const float va = __shfl(acc_a, m), vn = __shfl(acc_n, m);
        float v = 0.0f;
        if (col < 2 * sh.n_mat) v = (col & 1) ? vn : va;
        else if (col < n_par) v = (&sm.dd[0][0])[col - 2 * sh.n_mat];
        if (col < row_stride) prow[col] = v;
    }
}

// Two-stage FP64 column sums of partials[n_rows][stride] (stride a power of
// two <= 128, so 256 threads walking a row-aligned flat range always hit
// column t % stride).  Stage 1: block b sums rows [b*rpb, (b+1)*rpb) into
// stage1[b][stride]; stage 2: one block sums stage1's rows.  Every sum runs
// in a fixed order.
constexpr int kReduceThreads = 256;
constexpr int kReduceBlocks = 512;

template <typename T>
__device__ __forceinline__ void column_sums(const T *__restrict__ flat, int64_t len, int stride, double *out)
{
    __shared__ double s[kReduceThreads];
    double acc = 0.0;
    int64_t i = threadIdx.x;
    for (; i + 7 * kReduceThreads < len; i += 8 * kReduceThreads) {      // loads batched, adds in order
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = flat[i + k * kReduceThreads];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += (double)v[k];
    }
    for (; i < len; i += kReduceThreads) acc += (double)flat[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    if ((int)threadIdx.x < stride) {
        double v = 0.0;
        for (int k = threadIdx.x; k < kReduceThreads; k += stride) v += s[k];
        out[threadIdx.x] = v;
    }
}

// the gradients of an empty image: all zero
__global__ __launch_bounds__(kReduceThreads) void glint_bwd_zero_grads(float *ga, float *gn, float *gd, int n_mat,
                                                                       int n_light)
{
    const int i = threadIdx.x;
    if (i < n_mat) {
        ga[i] = 0.0f;
        gn[i] = 0.0f;
    }
    if (i < 3 * n_light) gd[i] = 0.0f;
}

// list_len (nullable): with the lit-pixel list, only the rows of the
// ceil(list_len / 64) chunks hold partial sums.
__global__ __launch_bounds__(kReduceThreads) void glint_bwd_reduce1(const float *partials, int64_t n_rows,
                                                                    const uint32_t *list_len, int stride,
                                                                    int64_t rpb, double *stage1)
{
    if (list_len) {
        const int64_t used = ((int64_t)list_len[0] + kWave - 1) / kWave;
        n_rows = used < n_rows ? used : n_rows;
    }
    const int64_t r0 = (int64_t)blockIdx.x * rpb;
    const int64_t r1 = r0 + rpb < n_rows ? r0 + rpb : n_rows;
    column_sums(partials + r0 * stride, r1 > r0 ? (r1 - r0) * stride : 0, stride,
                stage1 + (int64_t)blockIdx.x * stride);
}

__global__ __launch_bounds__(kReduceThreads) void glint_bwd_reduce2(const double *stage1, int n_blk, int stride,
                                                                    int n_mat, int n_par, float *g_alpha,
                                                                    float *g_lnN, float *g_dir)
{
    __shared__ double tot[128];
    column_sums(stage1, (int64_t)n_blk * stride, stride, tot);
    __syncthreads();
    const int c = threadIdx.x;
    if (c < n_par) {
        const float v = (float)tot[c];
        if (c < 2 * n_mat) {
            if (c & 1) g_lnN[c >> 1] = v; else g_alpha[c >> 1] = v;
        } else {
            g_dir[c - 2 * n_mat] = v;
        }
    }
}

static int64_t bwd_tiles(int32_t width, int32_t height)
{
    return tiles_of(width, height);
}

// ---------------------------------------------------------------------------
// Lit-pixel list for the adjoint: the pixels whose lit mask is non-zero, in
// raster order.  A segment is kLitSeg pixels of one row (the last one of a
// row shorter); segments are numbered in raster order.  A workgroup of
// kLitThreads threads handles one segment, each thread kLitPer consecutive
// pixels.
//   count:   lit pixels per segment
//   scan:    one workgroup turns the counts into offsets and the list length
//            (each thread a contiguous run of segments, loads issued 8 at a
//            time)
//   scatter: each segment writes its lit pixels' indices y*stride + x
// ---------------------------------------------------------------------------
constexpr int kLitThreads = 256;
constexpr int kLitPer = 4;
constexpr int kLitSeg = kLitThreads * kLitPer;
constexpr int kLitScan = 1024;

// this thread's lit flags (bit i: pixel x0 + i) in segment seg
__device__ __forceinline__ uint32_t lit_flags(const uint16_t *__restrict__ lit, int32_t width, int64_t stride,
                                              int32_t segs_x, int64_t seg, int64_t &y, int &x0)
{
    y = seg / segs_x;
    x0 = (int)(seg - y * segs_x) * kLitSeg + (int)threadIdx.x * kLitPer;
    uint32_t f = 0u;
#pragma unroll
    for (int i = 0; i < kLitPer; ++i)
        if (x0 + i < width && lit[y * stride + x0 + i] != 0) f |= 1u << i;
    return f;
}

// exclusive prefix of v over the workgroup's threads (in thread order) and the total
__device__ __forceinline__ uint32_t block_prefix(uint32_t v, uint32_t &total)
{
    __shared__ uint32_t wsum[kLitThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t incl = (uint32_t)wave_inclusive_sum((int)v);
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < kLitThreads / kWave; ++k) {
        before += k < w ? wsum[k] : 0u;
        total += wsum[k];
    }
    return before + incl - v;
}

__global__ __launch_bounds__(kLitThreads) void glint_lit_count(const uint16_t *__restrict__ lit, int32_t width,
                                                               int64_t stride, int32_t segs_x,
                                                               uint32_t *__restrict__ counts)
{
    int64_t y;
    int x0;
    const uint32_t f = lit_flags(lit, width, stride, segs_x, blockIdx.x, y, x0);
    uint32_t total;
    block_prefix((uint32_t)__popc(f), total);
    if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// n_dev (nullable): scan only the first ceil(n_dev[0] / 64) counts (the
// chunks of a list of n_dev[0] entries), at most n
__global__ __launch_bounds__(kLitScan) void glint_lit_scan(const uint32_t *__restrict__ counts, int64_t n,
                                                           uint32_t *__restrict__ offs, uint32_t *__restrict__ len,
                                                           const uint32_t *__restrict__ n_dev)
{
    constexpr int kScanWaves = kLitScan / kWave;
    __shared__ uint32_t ws[kScanWaves];
    const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
    if (n_dev) {
        const int64_t m = ((int64_t)n_dev[0] + kWave - 1) / kWave;
        n = m < n ? m : n;
    }
    const int64_t per = (n + kLitScan - 1) / kLitScan;
    const int64_t b0 = (int64_t)t * per < n ? (int64_t)t * per : n;
    const int64_t b1 = b0 + per < n ? b0 + per : n;
    uint32_t own = 0;
    int64_t i = b0;
    for (; i + 8 <= b1; i += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = counts[i + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) own += v[k];
    }
    for (; i < b1; ++i) own += counts[i];
    // exclusive prefix of the per-thread sums: DPP scan within the wave, then
    // the totals of the waves before this one
    const uint32_t incl = (uint32_t)wave_inclusive_sum((int)own);
    if (lane == kWave - 1) ws[w] = incl;
    __syncthreads();
    uint32_t pre = 0, total = 0;
#pragma unroll
    for (int k = 0; k < kScanWaves; ++k) {
        const uint32_t x = ws[k];
        total += x;
        pre += k < w ? x : 0u;
    }
    uint32_t run = pre + incl - own;
    i = b0;
    for (; i + 8 <= b1; i += 8) {
        uint32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = counts[i + k];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            offs[i + k] = run;
            run += v[k];
        }
    }
    for (; i < b1; ++i) {
        offs[i] = run;
        run += counts[i];
    }
    if (t == kLitScan - 1) len[0] = total;
}

__global__ __launch_bounds__(kLitThreads) void glint_lit_scatter(const uint16_t *__restrict__ lit, int32_t width,
                                                                 int64_t stride, int32_t segs_x,
                                                                 const uint32_t *__restrict__ offs,
                                                                 uint32_t *__restrict__ list)
{
    int64_t y;
    int x0;
    const uint32_t f = lit_flags(lit, width, stride, segs_x, blockIdx.x, y, x0);
    uint32_t total;
    uint32_t pos = offs[blockIdx.x] + block_prefix((uint32_t)__popc(f), total);
#pragma unroll
    for (int i = 0; i < kLitPer; ++i)
        if (f & (1u << i)) list[pos++] = (uint32_t)(y * stride + x0 + i);
}

static int row_stride_of(int n_par)
{
    int p = 1;
    while (p < n_par) p <<= 1;
    return p;
}

struct BwdLayout {
    size_t part_off, stage1_off, list_off, counts_off, offs_off, len_off, nb_off, uoff_off, nunits_off, bytes;
    int stride;
    int64_t rpb, n_blk, n_seg, n_chunks;
    int32_t segs_x;
};

// rows -> (rows per first-stage block, first-stage blocks)
static void reduce_shape(int64_t rows, int64_t &rpb, int64_t &n_blk)
{
    rpb = (rows + kReduceBlocks - 1) / kReduceBlocks;
    n_blk = rpb > 0 ? (rows + rpb - 1) / rpb : 0;
}

static BwdLayout bwd_layout(int32_t width, int32_t height, int n_par)
{
    BwdLayout L;
    const size_t a = 256;
    const int64_t tiles = bwd_tiles(width, height);
    const int64_t rows = tiles > kUnitGroups ? tiles : kUnitGroups;   // tiles, list chunks or unit workgroups
    L.stride = row_stride_of(n_par);
    reduce_shape(tiles, L.rpb, L.n_blk);
    L.part_off = (tile_order_bytes(width, height) + a - 1) / a * a;
    L.stage1_off = L.part_off + ((size_t)rows * L.stride * 4 + a - 1) / a * a;
    L.segs_x = (width + kLitSeg - 1) / kLitSeg;
    L.n_seg = (int64_t)L.segs_x * height;
    L.n_chunks = ((int64_t)width * height + kWave - 1) / kWave;
    L.list_off = L.stage1_off + ((size_t)kReduceBlocks * L.stride * 8 + a - 1) / a * a;
    L.counts_off = L.list_off + ((size_t)width * height * 4 + a - 1) / a * a;
    L.offs_off = L.counts_off + ((size_t)L.n_seg * 4 + a - 1) / a * a;
    L.len_off = L.offs_off + ((size_t)L.n_seg * 4 + a - 1) / a * a;
    L.nb_off = L.len_off + a;
    L.uoff_off = L.nb_off + ((size_t)L.n_chunks * 4 + a - 1) / a * a;
    L.nunits_off = L.uoff_off + ((size_t)L.n_chunks * 4 + a - 1) / a * a;
    L.bytes = L.nunits_off + a;
    return L;
}

}  // namespace glint

using namespace glint;

extern "C" {

size_t glint_backward_workspace_bytes(int32_t width, int32_t height, int32_t n_mat, int32_t n_light)
{
    if (width <= 0 || height <= 0 || n_mat < 1 || n_mat > kMaxMat || n_light < 0 || n_light > kMaxLight) return 0;
    return bwd_layout(width, height, 2 * n_mat + 3 * n_light).bytes;
}

int glint_shade_backward(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                         const glint_light *lights, int32_t n_light, const glint_params *params,
                         const float *grad_out_rgb, const uint16_t *lit_lights, const uint32_t *lit_probes,
                         float *grad_alpha, float *grad_ln_density, float *grad_light_dir, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    if (!params) return GLINT_ENULL;
    glint_params prm = *params;
    prm.rounding = 1;                            // the adjoint differentiates the relaxed counts
    Shared sh;
    int rc = prepare_shared(mats, n_mat, lights, n_light, &prm, sh);
    if (rc) return rc;
    if (!grad_alpha || !grad_ln_density || (n_light > 0 && !grad_light_dir)) return GLINT_ENULL;
    if ((reinterpret_cast<uintptr_t>(lit_lights) & 1u) != 0 || (reinterpret_cast<uintptr_t>(lit_probes) & 3u) != 0)
        return GLINT_EINVAL;
    ViewDesc vw;
    rc = make_view(gbuf, reinterpret_cast<float *>(const_cast<float *>(grad_out_rgb)), vw);
    if (rc) return rc;
    if (vw.alpha_px || vw.log10N_px) return GLINT_EUNSUPPORTED;
    const int n_par = 2 * n_mat + 3 * n_light;
    const int64_t tiles = (int64_t)vw.width * vw.height > 0 ? bwd_tiles(vw.width, vw.height) : 0;
    hipStream_t st = (hipStream_t)stream;
    if (tiles == 0) {
        // empty image: gradients are zero (a kernel, not a memset node, so
        // that the call stays safe to capture into a graph)
        hipLaunchKernelGGL(glint_bwd_zero_grads, dim3(1), dim3(kReduceThreads), 0, st, grad_alpha, grad_ln_density,
                           grad_light_dir, n_mat, n_light);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? GLINT_OK : set_hip_error(e);
    }
    if (tiles > 0x7fffffffLL) return GLINT_ESHAPE;
    const BwdLayout L = bwd_layout(vw.width, vw.height, n_par);
    if (!workspace) return GLINT_ENULL;
    if (workspace_bytes < L.bytes) return GLINT_ESHAPE;
    if ((uintptr_t)workspace & 7u) return GLINT_EINVAL;
    const int tiles_x = (int)tiles_x_of(vw.width);
    float *partials = (float *)((char *)workspace + L.part_off);
    double *stage1 = (double *)((char *)workspace + L.stage1_off);
    const uint32_t *list = nullptr, *list_len = nullptr;
    const int32_t *order = nullptr;
    int64_t grid = tiles;
    // list entries are y*stride + x in 32 bits
    const bool fits = (int64_t)vw.height * vw.stride <= 0xffffffffLL;
    if (lit_lights && lit_probes && n_light > 0 && fits) {
        // both masks: balanced units of (pixel, lit probe, lit light) items
        uint32_t *d_list = (uint32_t *)((char *)workspace + L.list_off);
        uint32_t *d_counts = (uint32_t *)((char *)workspace + L.counts_off);
        uint32_t *d_offs = (uint32_t *)((char *)workspace + L.offs_off);
        uint32_t *d_len = (uint32_t *)((char *)workspace + L.len_off);
        uint32_t *d_nb = (uint32_t *)((char *)workspace + L.nb_off);
        uint32_t *d_uoff = (uint32_t *)((char *)workspace + L.uoff_off);
        uint32_t *d_nunits = (uint32_t *)((char *)workspace + L.nunits_off);
        hipLaunchKernelGGL(glint_lit_count, dim3((unsigned)L.n_seg), dim3(kLitThreads), 0, st, lit_lights,
                           vw.width, vw.stride, L.segs_x, d_counts);
        hipLaunchKernelGGL(glint_lit_scan, dim3(1), dim3(kLitScan), 0, st, d_counts, L.n_seg, d_offs, d_len,
                           (const uint32_t *)nullptr);
        hipLaunchKernelGGL(glint_lit_scatter, dim3((unsigned)L.n_seg), dim3(kLitThreads), 0, st, lit_lights,
                           vw.width, vw.stride, L.segs_x, d_offs, d_list);
        const int64_t count_groups = std::min<int64_t>((L.n_chunks + kUnitWaves - 1) / kUnitWaves, 2048);
        hipLaunchKernelGGL(glint_unit_count, dim3((unsigned)count_groups), dim3(kWave * kUnitWaves), 0, st, vw, sh,
                           lit_lights, lit_probes, d_list, d_len, L.n_chunks, d_nb);
        hipLaunchKernelGGL(glint_lit_scan, dim3(1), dim3(kLitScan), 0, st, d_nb, L.n_chunks, d_uoff, d_nunits, d_len);
        hipLaunchKernelGGL(glint_bwd_unit_kernel, dim3(kUnitGroups), dim3(kWave), 0, st, vw, sh, grad_out_rgb,
                           lit_lights, lit_probes, d_list, d_len, d_uoff, d_nunits, partials, n_par, L.stride);
        int64_t rpb, n_blk;
        reduce_shape(kUnitGroups, rpb, n_blk);
        hipLaunchKernelGGL(glint_bwd_reduce1, dim3((unsigned)n_blk), dim3(kReduceThreads), 0, st, partials,
                           (int64_t)kUnitGroups, (const uint32_t *)nullptr, L.stride, rpb, stage1);
        hipLaunchKernelGGL(glint_bwd_reduce2, dim3(1), dim3(kReduceThreads), 0, st, stage1, (int)n_blk, L.stride,
                           n_mat, n_par, grad_alpha, grad_ln_density, grad_light_dir);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? GLINT_OK : set_hip_error(e);
    }
    if (lit_lights && fits) {
        uint32_t *d_list = (uint32_t *)((char *)workspace + L.list_off);
        uint32_t *d_counts = (uint32_t *)((char *)workspace + L.counts_off);
        uint32_t *d_offs = (uint32_t *)((char *)workspace + L.offs_off);
        uint32_t *d_len = (uint32_t *)((char *)workspace + L.len_off);
        hipLaunchKernelGGL(glint_lit_count, dim3((unsigned)L.n_seg), dim3(kLitThreads), 0, st, lit_lights,
                           vw.width, vw.stride, L.segs_x, d_counts);
        hipLaunchKernelGGL(glint_lit_scan, dim3(1), dim3(kLitScan), 0, st, d_counts, L.n_seg, d_offs, d_len,
                           (const uint32_t *)nullptr);
        hipLaunchKernelGGL(glint_lit_scatter, dim3((unsigned)L.n_seg), dim3(kLitThreads), 0, st, lit_lights,
                           vw.width, vw.stride, L.segs_x, d_offs, d_list);
        list = d_list;
        list_len = d_len;
        grid = ((int64_t)vw.width * vw.height + kWave - 1) / kWave;   // chunks beyond the list exit at once
    } else {
        rc = enqueue_tile_order(vw, sh, workspace, L.part_off, &order, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(glint_bwd_kernel, dim3((unsigned)grid), dim3(kWave), 0, st, vw, sh, grad_out_rgb, lit_lights,
                       lit_lights ? lit_probes : nullptr, list, list_len, tiles_x, order, (int32_t)tiles, partials,
                       n_par, L.stride);
    hipLaunchKernelGGL(glint_bwd_reduce1, dim3((unsigned)L.n_blk), dim3(kReduceThreads), 0, st, partials, tiles,
                       list_len, L.stride, L.rpb, stage1);
    hipLaunchKernelGGL(glint_bwd_reduce2, dim3(1), dim3(kReduceThreads), 0, st, stage1, (int)L.n_blk, L.stride,
                       n_mat, n_par, grad_alpha, grad_ln_density, grad_light_dir);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GLINT_OK : set_hip_error(e);
}

}  // extern "C"
