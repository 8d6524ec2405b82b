// glint_device.hpp -- device-side building blocks of per-pixel glint shading
// for CDNA4 (gfx950).  Internal header of the HIP library; not installed.
//
// Precision plan.  Every discrete decision of the method is taken from values
// whose error stays far below the 1e-5 decision margins:
//  * FP64 (full rate on CDNA4): footprint moments and |det J|, footprint
//    orientation, probe centres, the rotate/scale/skew into each grid's
//    simplex lattice (cell coordinates reach 1e4..1e6), the half vector and
//    its projection on the angular grid, 1 - cos^2 of the half vector.
//  * FP32: everything continuous after that (barycentric weights, p, gate
//    probabilities, Gaussian parameters, counts, BRDF) and the uniforms'
//    inverse CDF.  The gate is compared in exact integer form.
//  * integer (exact): texel keys and the hash.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glint {

constexpr int kMaxMat = 32;
constexpr int kMaxLight = 16;
constexpr int kWave = 64;
constexpr float kPiF = 3.14159265358979323846f;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Kernel-argument blocks (prepared by the host, passed by value)
// ---------------------------------------------------------------------------
struct DevMaterial {
    int32_t ndf;
    float alpha, R, log10N, F0;
    uint32_t root;            // hash state after absorbing the material seed
    double inv_micro;         // 1 / angular cell size
};

struct DevLight {
    double wo[3];             // unit direction toward the light (FP64 normalised)
    float rad[3];
    float inv_len;            // 1 / |raw direction| (for gradients w.r.t. the raw vector)
    int32_t ok;               // 0 when the raw direction has zero length
};

struct Shared {
    DevMaterial mats[kMaxMat];
    DevLight lights[kMaxLight];
    double cs[32][2];         // cos, sin of m pi / 32: every grid orientation up to ratio level 4
    int32_t n_mat, n_light, k_max, n_probe_max, rounding;
    const uint32_t *rng_tbl;  // random-number table variant: 2^b words (nullptr: hashed uniforms)
    uint32_t rng_mask;        // 2^b - 1
};

// The pixel that owns item q of a tile: the last p in 0..63 with off[p] <= q,
// for the non-decreasing item offsets of the tile's pixels (off[0] = 0),
// where `off` is this lane's offset (lane = pixel).  Two rounds of
// independent cross-lane reads (the 8-pixel block, then the pixel in it)
// instead of a six-step chain of dependent ones.  Every lane of the wave must
// be active.
__device__ __forceinline__ int item_pixel(int off, int q)
{
    int c = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) c += (__builtin_amdgcn_readlane(off, 8 * k) <= q) ? 1 : 0;
    const int b = 8 * c;
    int p = b;
#pragma unroll
    for (int i = 1; i < 8; ++i) p += (__shfl(off, b + i) <= q) ? 1 : 0;
    return p;
}

// Lane v moved by the DPP control CTRL within the rows of the mask ROWS;
// lanes whose source lies outside their 16-lane row, or in rows the mask
// leaves out, get 0.  Every lane of the wave must be active.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}

// inclusive prefix sum over the 64 lanes (all active): row shifts by 1, 2,
// 4, 8, then the row broadcasts 15 and 31
__device__ __forceinline__ int wave_inclusive_sum(int x)
{
    x += (int)dpp_mov<0x111, 0xf>((uint32_t)x);   // row_shr:1
    x += (int)dpp_mov<0x112, 0xf>((uint32_t)x);   // row_shr:2
    x += (int)dpp_mov<0x114, 0xf>((uint32_t)x);   // row_shr:4
    x += (int)dpp_mov<0x118, 0xf>((uint32_t)x);   // row_shr:8
    x += (int)dpp_mov<0x142, 0xa>((uint32_t)x);   // row_bcast:15 into rows 1 and 3
    x += (int)dpp_mov<0x143, 0xc>((uint32_t)x);   // row_bcast:31 into rows 2 and 3
    return x;
}

struct ViewDesc {
    int32_t width, height;
    int64_t stride;
    const float *u, *v, *dudx, *dvdx, *dudy, *dvdy, *nx, *ny, *nz, *wx, *wy, *wz;
    const int32_t *mat;
    const float *alpha_px, *log10N_px;
    float *out;
    const float *tx, *ty, *tz;   // optional supplied tangent (all three or none)
};

struct DebugPlanes {
    uint32_t *flags;
    int32_t *n_probe, *level;
    uint32_t *cell, *key_sum, *akey_sum, *theta_sum, *count_sum, *n_open, *n_gate, *n_live;
    float *b_light;
    uint32_t *n_live_small, *n_lit, *n_live_lit;
    // sampled per-texel dump: slot plane, capacity, probes per slot, arrays
    const int32_t *dump_slot;
    int32_t dump_cap, dump_probes;
    uint32_t *dump_key;
    float *dump_beta;
    uint32_t *dump_theta;
    float *dump_count;
};

enum : uint32_t {
    F_SHADED = 1u, F_CLAMP_RATIO = 2u, F_CLAMP_P = 4u, F_BAD_INPUT = 8u,
    F_BACKFACING = 16u, F_SKIPPED = 32u, F_BAD_MAT = 64u
};

// ---------------------------------------------------------------------------
// Per-texel random numbers.  H(h, w) = fmix32((h ^ w) + golden), fmix32 the
// MurmurHash3 finaliser; chains absorb one key word per step.
// ---------------------------------------------------------------------------
// (host and device: the host derives each material's root state with it)
__host__ __device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint32_t hstep(uint32_t h, uint32_t w)
{
    return fmix32((h ^ w) + 0x9E3779B9u);
}

// H(h, w) without fmix32's last step x ^= x >> 16.  That step keeps the top
// 16 bits and is the identity when they are zero, so for t < 2^16:
// H(h, w) <= t  <=>  hstep_head(h, w) <= t.
__device__ __forceinline__ uint32_t hstep_head(uint32_t h, uint32_t w)
{
    uint32_t x = (h ^ w) + 0x9E3779B9u;
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    return x;
}

constexpr uint32_t kRootSalt = 0x243F6A88u;     // material seed chain start
constexpr uint32_t kAngularSalt = 0x13198A2Eu;  // angular key chain start

__device__ __forceinline__ uint32_t node_word(int l, int k, int m)
{
    return (uint32_t)(l + 1024) | ((uint32_t)k << 11) | ((uint32_t)m << 14);
}

__device__ __forceinline__ uint32_t angular_word(int ai, int aj, int s)
{
    return ((uint32_t)(ai + 16384) & 0x7FFFu) | (((uint32_t)(aj + 16384) & 0x7FFFu) << 15) |
           ((uint32_t)s << 30);
}

// Standard normal inverse CDF of the uniform (2 (h >> 9) + 1) 2^-24 that the
// hash word h stands for.  Two-region erfinv approximation after Giles
// (2011) with coefficients fitted for this library (fit_ndtri.py):
// max relative error 3.1e-7 over all 2^23 uniforms.  x = 2q - 1, 1 - x and
// 1 + x are exact in FP32.
__device__ __forceinline__ float ndtri_bits(uint32_t h)
{
    const int k = (int)(h >> 9);
    const float x = (float)(2 * k + 1 - 8388608) * 0x1p-23f;
    const float omx = (float)(16777215 - 2 * k) * 0x1p-23f;   // 1 - x
    const float opx = (float)(2 * k + 1) * 0x1p-23f;          // 1 + x
    // v_log_f32 (log2, <= 1 ulp): the polynomial depends weakly on w in the
    // centre and like sqrt(w) in the tails, so ulp-level errors in w stay far
    // below the count margins
    float w = -0.69314718055994531f * __builtin_amdgcn_logf(omx * opx);
    float p;
    if (w < 5.0f) {
        const float s = w - 2.5f;
        p = 2.798955556e-08f;
        p = fmaf(p, s, 3.430734239e-07f);
        p = fmaf(p, s, -3.522236511e-06f);
        p = fmaf(p, s, -4.389634341e-06f);
        p = fmaf(p, s, 2.185773774e-04f);
        p = fmaf(p, s, -1.253729803e-03f);
        p = fmaf(p, s, -4.177678842e-03f);
        p = fmaf(p, s, 2.466407418e-01f);
        p = fmaf(p, s, 1.501409411e+00f);
    } else {
        const float s = __builtin_amdgcn_sqrtf(w) - 3.0f;
        p = -2.158486895e-04f;
        p = fmaf(p, s, 1.057877307e-04f);
        p = fmaf(p, s, 1.370809623e-03f);
        p = fmaf(p, s, -3.677487373e-03f);
        p = fmaf(p, s, 5.730178207e-03f);
        p = fmaf(p, s, -7.621666417e-03f);
        p = fmaf(p, s, 9.440163150e-03f);
        p = fmaf(p, s, 1.001674056e+00f);
        p = fmaf(p, s, 2.832976818e+00f);
    }
    return 1.41421356237309505f * p * x;
}

// ---------------------------------------------------------------------------
// Per-pixel setup: footprint (Sec. 5.1), probe count (Sec. 4.2), the grid
// nodes of the tetrahedron enclosing (area, ratio, orientation) (Eq. 13,
// Fig. 4, Sec. 6.1) and the distributed weights (Eq. 10).
// ---------------------------------------------------------------------------
struct Pixel {
    uint32_t flags;
    int mat;
    float alpha, N;            // roughness, flakes per unit UV area
    double n[3], wi[3];
    double rc, rs;             // tangent frame: rotation of the basis of n (1, 0 without a tangent)
    double cos_i;
    double u, v, P;            // uv and |det J|
    double ex, ey;             // sigma0 * major axis direction
    int npr;
    int n_nodes;
    int nl[4], nk[4], nm[4];
    float nw[4];
    int level;
    uint32_t cell;
};

__device__ __forceinline__ bool finitef(float x) { return (__float_as_uint(x) & 0x7f800000u) != 0x7f800000u; }

// FP64 1/sqrt(x) and 1/x for finite x > 0 (x != 0 for the reciprocal): the
// hardware seed (v_rsq_f64 / v_rcp_f64, within 6e-8 relative on gfx950)
// refined by one Newton step, which squares the error: within 5e-15
// relative, at a quarter of the cost of the IEEE sequences.  Used where such
// an error cannot decide anything exactly (every decision downstream has a
// boundary margin of 1e-5 in its own units).
__device__ __forceinline__ double rsqrt_d(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);          // 1 - x y^2
    return fma(0.5 * y, e, y);
}

__device__ __forceinline__ double rcp_d(double x)
{
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

// FP64 normalisation of an FP32 input vector (identical wherever it is used)
__device__ __forceinline__ bool normalize_in(float x, float y, float z, double out[3])
{
    double l2 = (double)x * x + (double)y * y + (double)z * z;
    if (!(l2 > 0.0)) return false;          // FP32 inputs: 0 < l2 < 4e77, rsq in range
    const double il = rsqrt_d(l2);
    out[0] = x * il; out[1] = y * il; out[2] = z * il;
    return true;
}

// log2 x for x >= 1 (a footprint's ratio), exact at powers of two and
// within about 1e-15 elsewhere: x = m 2^e with m in [1/sqrt 2, sqrt 2) and
// log2 m = (2 / ln 2) atanh(s), s = (m - 1)/(m + 1), |s| <= 0.1716, from the
// odd series of atanh through s^21 (truncation below 1e-18 relative)
__device__ __forceinline__ double log2_ratio(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) { m *= 2.0; e -= 1; }
    const double s = (m - 1.0) * rcp_d(m + 1.0);
    const double s2 = s * s;
    double t = 1.0 / 21.0;
    t = fma(t, s2, 1.0 / 19.0);
    t = fma(t, s2, 1.0 / 17.0);
    t = fma(t, s2, 1.0 / 15.0);
    t = fma(t, s2, 1.0 / 13.0);
    t = fma(t, s2, 1.0 / 11.0);
    t = fma(t, s2, 1.0 / 9.0);
    t = fma(t, s2, 1.0 / 7.0);
    t = fma(t, s2, 1.0 / 5.0);
    t = fma(t, s2, 1.0 / 3.0);
    t = fma(t, s2, 1.0);
    return (double)e + (2.88539008177792681472 * s) * t;
}

// The tangent frame (t, b, n) of the angular grid (Eq. 14).  The orthonormal
// basis (t0, b0, n) of n after Duff et al. (2017) is kept in implicit form:
// with s = sign(n_z) and a = -1/(s + n_z) its axes are
// t0 = (1 + s a nx^2, s a nx ny, -s nx) and b0 = (a nx ny, s + a ny^2, -ny),
// so for any w, with d = a (nx wx + ny wy) - wz:
//   <t0, w> = wx + s nx d,   <b0, w> = s wy + ny d.
// A supplied tangent (reading of Sec. 5.2: made orthogonal to n and
// normalised, b = n x t) lies in the span of t0 and b0, so the frame is t0, b0
// turned about n by the unit rotation (rc, rs): t = rc t0 + rs b0 and
// b = n x t = -rs t0 + rc b0 (the basis is right-handed).  Without a tangent
// (rc, rs) = (1, 0), and the rotation reproduces <t0, w>, <b0, w> exactly.
struct ViewFrame {
    double a, s, snx;          // a, s = sign(n_z), s n_x
    double rc, rs;             // rotation of (t0, b0) into (t, b)
    double cos_i, wt, wb;      // <n, wi>, <wi, t>, <wi, b>
};

// <t, w> and <b, w> from nw = nx wx + ny wy
__device__ __forceinline__ void frame_dots(const double n[3], const ViewFrame &f, const double w[3], double nw,
                                           double &tw, double &bw)
{
    const double d = f.a * nw - w[2];
    const double t0 = fma(f.snx, d, w[0]);
    const double b0 = fma(n[1], d, f.s * w[1]);
    tw = fma(f.rs, b0, f.rc * t0);
    bw = fma(f.rc, b0, -(f.rs * t0));
}

// the axes themselves (the adjoint's light-direction gradient)
__device__ __forceinline__ void frame_axes(const double n[3], const ViewFrame &f, double t[3], double b[3])
{
    const double bb = n[0] * n[1] * f.a;
    const double t0[3] = {1.0 + f.snx * n[0] * f.a, f.s * bb, -f.snx};
    const double b0[3] = {bb, f.s + n[1] * n[1] * f.a, -n[1]};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        t[c] = fma(f.rs, b0[c], f.rc * t0[c]);
        b[c] = fma(f.rc, b0[c], -(f.rs * t0[c]));
    }
}

__device__ __forceinline__ void view_frame(const double n[3], const double wi[3], double rc, double rs, ViewFrame &f)
{
    f.s = copysign(1.0, n[2]);
    f.a = -rcp_d(f.s + n[2]);                      // |s + n_z| >= 1
    f.snx = f.s * n[0];
    f.rc = rc;
    f.rs = rs;
    f.cos_i = n[0] * wi[0] + n[1] * wi[1] + n[2] * wi[2];
    frame_dots(n, f, wi, n[0] * wi[0] + n[1] * wi[1], f.wt, f.wb);
}

// The rotation (rc, rs) of a supplied tangent (FP32 inputs tin) about the unit
// normal n: rc = <tin, t0>/q, rs = <tin, b0>/q with q the length of tin's
// component in the tangent plane.  A tangent within about 1e-3 rad of n
// (sin^2 of the angle below 1e-6, the reading's threshold) or of zero length
// defines no frame: returns false (invalid input).
constexpr double kTangentMinSin2 = 1e-6;
__device__ __forceinline__ bool tangent_rotation(const double n[3], float tx, float ty, float tz, double &rc,
                                                 double &rs)
{
    ViewFrame f;
    f.s = copysign(1.0, n[2]);
    f.a = -rcp_d(f.s + n[2]);
    f.snx = f.s * n[0];
    f.rc = 1.0;
    f.rs = 0.0;
    const double t[3] = {tx, ty, tz};
    double c, sn;
    frame_dots(n, f, t, n[0] * t[0] + n[1] * t[1], c, sn);
    const double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];   // exact: products of FP32 values
    const double q2 = c * c + sn * sn;
    if (!(tt > 0.0) || !(q2 >= kTangentMinSin2 * tt)) return false;
    const double iq = rsqrt_d(q2);
    rc = c * iq;
    rs = sn * iq;
    return true;
}

// atan2(y, x) in FP64 within about 1e-15 rad (the footprint orientation's
// decisions have margins of 1e-5 cells): the ratio of the smaller to the
// larger of |y|, |x| (t <= 1), reduced to |t'| <= tan(pi/8) by
// atan t = pi/4 + atan((t - 1)/(t + 1)) above tan(pi/8), then the odd Taylor
// series of atan through t'^37 (truncation below 1e-16), and the octant
// restored.  Zero y gives exactly 0 or pi (x >= +0 or not), zero x exactly
// +-pi/2, as the C library does; the series' coefficients are uniform
// constants (scalar registers), unlike the library's table.
__device__ __forceinline__ double atan2_d(double y, double x)
{
    const double ax = fabs(x), ay = fabs(y);
    const bool swap = ay > ax;
    const double num = swap ? ax : ay, den = swap ? ay : ax;
    double t = den > 0.0 ? num * rcp_d(den) : 0.0;
    const bool big = t > 0.41421356237309503;
    if (big) t = (t - 1.0) * rcp_d(t + 1.0);
    const double t2 = t * t;
    double q = 1.0 / 37.0;
#pragma unroll
    for (int k = 17; k >= 0; --k) q = fma(q, -t2, 1.0 / (double)(2 * k + 1));
    double a = fma(t, q, big ? 0.78539816339744831 : 0.0);
    if (swap) a = 1.5707963267948966 - a;
    if (x < 0.0 || (x == 0.0 && signbit(x))) a = 3.1415926535897932 - a;
    if (ay == 0.0) a = (x < 0.0 || (x == 0.0 && signbit(x))) ? 3.1415926535897932 : 0.0;
    return signbit(y) ? -a : a;
}

template <bool DEBUG>
__device__ __forceinline__ void setup_pixel(const ViewDesc &vw, int64_t idx, const Shared &sh, Pixel &px)
{
    px.flags = 0;
    px.npr = 0;
    px.n_nodes = 0;
    px.level = 0;
    px.cell = 0;
    const int mat = vw.mat ? vw.mat[idx] : 0;
    px.mat = mat;
    if (mat < 0) { px.flags = F_SKIPPED; return; }
    if (mat >= sh.n_mat) { px.flags = F_BAD_MAT; return; }
    const DevMaterial &M = sh.mats[mat];
    const float fu = vw.u[idx], fv = vw.v[idx];
    const float dux = vw.dudx[idx], dvx = vw.dvdx[idx], duy = vw.dudy[idx], dvy = vw.dvdy[idx];
    const float fnx = vw.nx[idx], fny = vw.ny[idx], fnz = vw.nz[idx];
    const float fwx = vw.wx[idx], fwy = vw.wy[idx], fwz = vw.wz[idx];
    const float alpha = vw.alpha_px ? vw.alpha_px[idx] : M.alpha;
    const float l10 = vw.log10N_px ? vw.log10N_px[idx] : M.log10N;
    const float ftx = vw.tx ? vw.tx[idx] : 0.0f, fty = vw.tx ? vw.ty[idx] : 0.0f, ftz = vw.tx ? vw.tz[idx] : 0.0f;
    const int fin = (int)finitef(fu) & (int)finitef(fv) & (int)finitef(dux) & (int)finitef(dvx) &
                    (int)finitef(duy) & (int)finitef(dvy) & (int)finitef(fnx) & (int)finitef(fny) &
                    (int)finitef(fnz) & (int)finitef(fwx) & (int)finitef(fwy) & (int)finitef(fwz) &
                    (int)finitef(alpha) & (int)finitef(l10) & (int)finitef(ftx) & (int)finitef(fty) &
                    (int)finitef(ftz);
    if (!fin || !(alpha > 0.0f)) { px.flags = F_BAD_INPUT; return; }
    px.alpha = alpha;
    px.N = exp10f(l10);
    // normal and view, FP64 normalised
    if (!normalize_in(fnx, fny, fnz, px.n) || !normalize_in(fwx, fwy, fwz, px.wi)) {
        px.flags = F_BAD_INPUT;
        return;
    }
    // the angular grid's frame (Eq. 14): the supplied tangent, else the basis of n
    px.rc = 1.0;
    px.rs = 0.0;
    if (vw.tx && !tangent_rotation(px.n, ftx, fty, ftz, px.rc, px.rs)) {
        px.flags = F_BAD_INPUT;
        return;
    }
    // footprint: J J^T moments and |det J| in FP64 (products of FP32 are exact)
    const double a = (double)dux * dux + (double)duy * duy;
    const double b = (double)dux * dvx + (double)duy * dvy;
    const double c = (double)dvx * dvx + (double)dvy * dvy;
    const double P = fabs((double)dux * dvy - (double)duy * dvx);
    if (!(P > 0.0) || !(P < 1.0e300)) { px.flags = F_BAD_INPUT; return; }
    px.cos_i = px.n[0] * px.wi[0] + px.n[1] * px.wi[1] + px.n[2] * px.wi[2];
    if (!(px.cos_i > 0.0)) { px.flags = F_BACKFACING; return; }
    const double hd = 0.5 * (a - c);
    const double R = sqrt(hd * hd + b * b);
    const double s0sq = 0.5 * (a + c) + R;
    double r = s0sq / P;
    if (r < 1.0) r = 1.0;
    double phi = 0.5 * atan2_d(2.0 * b, a - c);
    if (phi < 0.0) phi += kPi;
    // sigma0 (cos phi, sin phi): the eigenvector of J J^T for sigma0^2 in its
    // well-conditioned form, (hd + R, b) or (b, R - hd), turned so that
    // sin phi >= 0 (phi in [0, pi)); an isotropic footprint takes phi = 0
    double vx = hd >= 0.0 ? hd + R : b, vy = hd >= 0.0 ? b : R - hd;
    if (vy < 0.0) { vx = -vx; vy = -vy; }
    const double vv = vx * vx + vy * vy;
    if (!(vv > 0.0)) { vx = 1.0; vy = 0.0; }
    const double sc = s0sq * rsqrt_d(s0sq) * (vv > 0.0 ? rsqrt_d(vv) : 1.0);
    px.u = fu; px.v = fv; px.P = P;
    px.ex = sc * vx;
    px.ey = sc * vy;
    // sub-footprints along the major axis when r exceeds the family's 2^K
    const int K = sh.k_max;
    const double rmax = (double)(1 << K);
    int npr = (int)ceil(r / rmax);
    if (npr < 1) npr = 1;
    if (npr > sh.n_probe_max) npr = sh.n_probe_max;
    px.npr = npr;
    const double Pk = npr > 1 ? P / npr : P;
    double rk = npr > 1 ? r / npr : r;
    if (rk > rmax) { rk = rmax; px.flags |= F_CLAMP_RATIO; }
    // area level (Eq. 13): Pk = fr 2^ex exactly, l = ex - 1, top weight ts (Eq. 10)
    int ex;
    const double fr = frexp(Pk, &ex);
    const int l = ex - 1;
    const double ts = 2.0 * fr - 1.0;
    px.level = l;
    // ratio / orientation cell (Fig. 4): ring kap holds 2^(kap+1) orientations.
    // FP64 here: small barycentric weights keep their relative precision.
    int tk[3], tm[3];
    double lam[3];
    int nv;
    int kap = 0, j = 0, tri = 0;
    if (K == 0) {
        nv = 1; tk[0] = 0; tm[0] = 0; lam[0] = 1.0;
        tk[1] = tk[2] = 0; tm[1] = tm[2] = 0; lam[1] = lam[2] = 0.0;
    } else {
        double rho = log2_ratio(rk);
        rho = fmin(fmax(rho, 0.0), (double)K);
        kap = min((int)floor(rho), K - 1);
        const double u = rho - (double)kap;
        const int M = 1 << (kap + 1);
        // phi / (pi / M) with pi / M = pi 2^-(kap+1) exact: the scaled quotient
        // phi / pi (exact boundary hits reproduce)
        const double q = ldexp(phi / kPi, kap + 1);
        j = (int)floor(q);
        j = max(0, min(j, M - 1));
        const double t = q - (double)j;
        const int jn = (j + 1) & (M - 1);
        const int o2 = (2 * j + 2) & (2 * M - 1);
        // pentagon (u,t): I0=(0,0) I1=(0,1) O0=(1,0) O1=(1,1/2) O2=(1,1), three triangles (Fig. 5)
        if (t <= 0.5 * u) {
            tri = 0;
            tk[0] = kap; tm[0] = j; lam[0] = 1.0 - u;
            tk[1] = kap + 1; tm[1] = 2 * j; lam[1] = u - 2.0 * t;
            tk[2] = kap + 1; tm[2] = 2 * j + 1; lam[2] = 2.0 * t;
        } else if (t >= 1.0 - 0.5 * u) {
            tri = 2;
            tk[0] = kap; tm[0] = jn; lam[0] = 1.0 - u;
            tk[1] = kap + 1; tm[1] = o2; lam[1] = u - 2.0 * (1.0 - t);
            tk[2] = kap + 1; tm[2] = 2 * j + 1; lam[2] = 2.0 * (1.0 - t);
        } else {
            tri = 1;
            tk[0] = kap; tm[0] = j; lam[0] = 1.0 - t - 0.5 * u;
            tk[1] = kap; tm[1] = jn; lam[1] = t - 0.5 * u;
            tk[2] = kap + 1; tm[2] = 2 * j + 1; lam[2] = u;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lam[i] = fmax(lam[i], 0.0);
            if (tk[i] == 0) tm[i] = 0;      // the isotropic grid has no orientation
        }
        nv = 3;
    }
    // merge coincident grids (only ring 0 of triangle I0-I1-O1 can coincide),
    // then order by key (k, m): a 3-element sorting network on registers
    int k0 = tk[0], k1 = tk[1], k2 = tk[2], m0 = tm[0], m1 = tm[1], m2 = tm[2];
    double l0 = lam[0], l1 = lam[1], l2 = lam[2];
    int D = nv;
    if (nv == 3 && k0 == k1 && m0 == m1) { l0 += l1; k1 = k2; m1 = m2; l1 = l2; D = 2; }
    if (D == 1) { k1 = k2 = 255; m1 = m2 = 0; l1 = l2 = 0.0; }
    if (D == 2) { k2 = 255; m2 = 0; l2 = 0.0; }
#define GLINT_CSWAP(ka, ma, la, kb, mb, lb)                                      \
    if ((ka) * 64 + (ma) > (kb) * 64 + (mb)) {                                   \
        int _k = ka; ka = kb; kb = _k; int _m = ma; ma = mb; mb = _m;            \
        double _l = la; la = lb; lb = _l;                                        \
    }
    GLINT_CSWAP(k0, m0, l0, k1, m1, l1)
    GLINT_CSWAP(k1, m1, l1, k2, m2, l2)
    GLINT_CSWAP(k0, m0, l0, k1, m1, l1)
#undef GLINT_CSWAP
    // prism -> tetrahedron: top-level mass ts goes to the highest keys first
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    int pivot;
    {
        double rem = ts;
        if (D == 3) {
            if (rem <= l2) { t2 = rem; pivot = 2; }
            else {
                t2 = l2; rem -= l2;
                if (rem <= l1) { t1 = rem; pivot = 1; }
                else { t1 = l1; rem -= l1; t0 = fmin(rem, l0); pivot = 0; }
            }
        } else if (D == 2) {
            if (rem <= l1) { t1 = rem; pivot = 1; }
            else { t1 = l1; rem -= l1; t0 = fmin(rem, l0); pivot = 0; }
        } else {
            t0 = fmin(rem, l0); pivot = 0;
        }
    }
    // tetrahedron vertices: bottoms of sorted[0..pivot], tops of sorted[pivot..D-1]
    const int n = D + 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const bool bottom = v <= pivot;
        const int src = bottom ? v : v - 1;
        const int kk = src == 0 ? k0 : (src == 1 ? k1 : k2);
        const int mmv = src == 0 ? m0 : (src == 1 ? m1 : m2);
        const double ll = src == 0 ? l0 : (src == 1 ? l1 : l2);
        const double tt = src == 0 ? t0 : (src == 1 ? t1 : t2);
        px.nl[v] = bottom ? l : l + 1;
        px.nk[v] = v < n ? kk : 0;
        px.nm[v] = v < n ? mmv : 0;
        px.nw[v] = v < n ? (float)(bottom ? ll - tt : tt) : 0.0f;
    }
    px.n_nodes = n;
    if (DEBUG)
        px.cell = (uint32_t)kap | ((uint32_t)j << 3) | ((uint32_t)tri << 9) | ((uint32_t)pivot << 11) |
                  ((uint32_t)D << 13) | ((uint32_t)n << 15);
    px.flags |= F_SHADED;
}

// Per-pixel record staged in LDS for the (pixel, probe) items: everything an
// item needs that does not depend on the probe (48 bytes).
//   pk     n_pr (bits 0-6) | node count (7-9) | material (10-14) | l + 1024 (15-25)
//   nd[2]  per node 9 bits, two nodes per word at bits 0 and 16:
//          top level (bit 0: level l + 1) | k << 1 | m << 4
// The bottom area level l lies in [-300, 256] for FP32 derivatives (|det J|
// is a product of two FP32 values), so l + 1024 takes 11 bits.
struct PixelRec {
    float ex, ey;              // sigma0 * major axis direction, rounded to FP32 (every kernel places the
                               // probes from these same values)
    uint32_t pk;
    float alpha, kpx, lam_i;   // roughness, D(n)/(R N P 4 <wi,n>), Smith Lambda of the view
    uint32_t nd[2];
    float ng[4];               // trials per node, w N 2^l (Eq. 10)
};

__device__ __forceinline__ int rec_npr(const PixelRec &R) { return (int)(R.pk & 0x7fu); }
__device__ __forceinline__ int rec_nodes(const PixelRec &R) { return (int)((R.pk >> 7) & 7u); }
__device__ __forceinline__ int rec_mat(const PixelRec &R) { return (int)((R.pk >> 10) & 31u); }

// key word (l + 1024) | k << 11 | m << 14 of node g
__device__ __forceinline__ uint32_t rec_node_word(const PixelRec &R, int g)
{
    const uint32_t d = (R.nd[g >> 1] >> ((g & 1) * 16)) & 0x1ffu;
    return (((R.pk >> 15) & 0x7ffu) + (d & 1u)) | (((d >> 1) & 7u) << 11) | ((d >> 4) << 14);
}

// ---------------------------------------------------------------------------
// Simplex lattice of grid node (l, k, m) around point c (Eq. 12 read as
// rotate-then-scale, Sec. 6.2 simplex grid): three vertices and barycentrics.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow2_neg_half(int e)   // 2^(-e/2)
{
    const double ir2 = 0.70710678118654752440;
    const int h = e >> 1;                 // floor(e/2): 2^(-e/2) = 2^-h (e even), 2^-h / sqrt 2 (e odd)
    return (e & 1) ? ldexp(ir2, -h) : ldexp(1.0, -h);
}

__device__ __forceinline__ void simplex_locate(double cx, double cy, int l, int k, int m, const Shared &sh,
                                               int vi[3], int vj[3], float beta[3])
{
    const int mi = k ? (m << (4 - k)) : 0;
    const double cph = sh.cs[mi][0], sph = sh.cs[mi][1];
    const double qx = cph * cx + sph * cy;
    const double qy = -sph * cx + cph * cy;
    const double x = qx * pow2_neg_half(l + k);
    const double y = qy * pow2_neg_half(l - k);
    const double Lx = x + 0.5 * y, Ly = y;
    const double fi = floor(Lx), fj = floor(Ly);
    const double f = Lx - fi, g = Ly - fj;
    const int i = (int)fi, j = (int)fj;
    if (f >= g) {
        vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j; vi[2] = i + 1; vj[2] = j + 1;
        beta[0] = (float)(1.0 - f); beta[1] = (float)(f - g); beta[2] = (float)g;
    } else {
        vi[0] = i; vj[0] = j; vi[1] = i; vj[1] = j + 1; vi[2] = i + 1; vj[2] = j + 1;
        beta[0] = (float)(1.0 - g); beta[1] = (float)(g - f); beta[2] = (float)f;
    }
}

// v_rcp_f32 (1 ulp): the relative error of every quotient below stays ~1e-7
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }

// log(1 - p) for p in [0, 1): atanh series 2s(1 + s^2/3 + ... + s^8/9) with
// s = -p/(2 - p) for p <= 1/4 (truncation < 4e-10 relative), hardware log2 of
// 1 - p above (|log(1-p)| > 0.28 there).  Relative error ~3e-7.
__device__ __forceinline__ float log1m(float p)
{
    const float s = -p * rcpf(2.0f - p);
    const float s2 = s * s;
    float t = fmaf(s2, 1.0f / 9.0f, 1.0f / 7.0f);
    t = fmaf(t, s2, 1.0f / 5.0f);
    t = fmaf(t, s2, 1.0f / 3.0f);
    t = fmaf(t, s2, 1.0f);
    const float small = 2.0f * s * t;
    const float large = 0.69314718055994531f * __builtin_amdgcn_logf(1.0f - p);
    return p <= 0.25f ? small : large;
}

// 1 - exp(y) for y <= 0: Taylor series to y^7 for |y| <= 1/4 (truncation
// < 4e-10 relative), 1 - 2^(y log2 e) below (result > 0.22).  ~2e-7 relative.
__device__ __forceinline__ float one_minus_exp(float y)
{
    float t = fmaf(y, 1.0f / 5040.0f, 1.0f / 720.0f);
    t = fmaf(t, y, 1.0f / 120.0f);
    t = fmaf(t, y, 1.0f / 24.0f);
    t = fmaf(t, y, 1.0f / 6.0f);
    t = fmaf(t, y, 0.5f);
    t = fmaf(t, y, 1.0f);
    const float small = -y * t;
    const float large = 1.0f - __builtin_amdgcn_exp2f(y * 1.4426950408889634f);
    return y >= -0.25f ? small : large;
}

// Smith Lambda of the NDF for a direction with cos theta = c, 1 - c^2 = s2
__device__ __forceinline__ float smith_lambda(int ndf, float alpha, float c, float s2)
{
    if (s2 <= 0.0f) return 0.0f;
    const float tan2 = s2 * rcpf(c * c);
    if (ndf == 0) return 0.5f * (-1.0f + __builtin_amdgcn_sqrtf(1.0f + alpha * alpha * tan2));
    const float a = rcpf(alpha * __builtin_amdgcn_sqrtf(tan2));
    return 0.5f * (erff(a) - 1.0f) + expf(-a * a) / (2.0f * a * 1.7724538509055160f);
}

// p = min(1, R D(h)/D(n)) (Eq. 4) from cos^2 and 1 - cos^2 of the half vector
__device__ __forceinline__ float success_prob(int ndf, float alpha, float R, float c2, float s2, bool &clamped)
{
    const float a2 = alpha * alpha;
    float ratio;
    if (ndf == 0) {
        const float d = s2 + c2 * a2;          // (n.h)^2 (a^2 - 1) + 1, cancellation-free
        ratio = (a2 * a2) * rcpf(d * d);
    } else {
        ratio = expf(-(s2 * rcpf(c2 * a2))) * rcpf(c2 * c2);
    }
    float p = R * ratio;
    clamped = p > 1.0f;
    return clamped ? 1.0f : p;
}

// Everything one light needs at one pixel (shared by the forward and the
// adjoint so that both take identical decisions).  The half vector
// h = (wi + wo)/|wi + wo| of the unit directions enters only through dot
// products: |wi + wo|^2 = 2 (1 + <wi,wo>), <n,h> = (<n,wi> + <n,wo>)/|wi + wo|,
// <wi,h> = (1 + <wi,wo>)/|wi + wo| and likewise for the frame axes.
struct LightEval {
    double ihl;                // 1 / |wi + wo|
    double wiwo;               // <wi, wo>
    double cos_o, ch;          // <n, wo>, <n, h>
    float p;                   // success probability (Eq. 4)
    bool pclamp;
    int ai, aj;                // angular cell (lower-left texel)
    float fx, fy, gx, gy;      // bilinear fractions and their complements
    float F, lam_o;            // Schlick Fresnel, Smith Lambda of wo (light_brdf; needed only with an open gate)
};

__device__ __forceinline__ bool eval_light(const double n[3], const double wi[3], float alpha, const DevLight &L,
                                           const DevMaterial &M, const ViewFrame &f, LightEval &e)
{
    if (!L.ok) return false;
    const double nw = n[0] * L.wo[0] + n[1] * L.wo[1];
    e.cos_o = nw + n[2] * L.wo[2];
    if (!(e.cos_o > 0.0)) return false;
    const double wiwo = wi[0] * L.wo[0] + wi[1] * L.wo[1] + wi[2] * L.wo[2];
    e.wiwo = wiwo;
    const double hh = 2.0 + 2.0 * wiwo;
    if (!(hh > 0.0)) return false;
    const double ihl = rsqrt_d(hh);
    e.ihl = ihl;
    e.ch = (f.cos_i + e.cos_o) * ihl;
    e.p = success_prob(M.ndf, alpha, M.R, (float)(e.ch * e.ch), (float)(1.0 - e.ch * e.ch), e.pclamp);
    // angular grid over the projected half vector (Eq. 14)
    const double sc = ihl * M.inv_micro;
    double tw, bw;
    frame_dots(n, f, L.wo, nw, tw, bw);
    const double ax = (f.wt + tw) * sc - 0.5;
    const double ay = (f.wb + bw) * sc - 0.5;
    const double fax = floor(ax), fay = floor(ay);
    e.ai = (int)fax; e.aj = (int)fay;
    // bilinear fractions; both complements from FP64 so small weights stay accurate
    e.fx = (float)(ax - fax); e.fy = (float)(ay - fay);
    e.gx = (float)(fax + 1.0 - ax); e.gy = (float)(fay + 1.0 - ay);
    return true;
}

// Schlick Fresnel and Smith Lambda of the light direction (Eq. 2)
__device__ __forceinline__ void light_brdf(const DevMaterial &M, float alpha, LightEval &e)
{
    const float om = (float)(1.0 - (1.0 + e.wiwo) * e.ihl);
    const float om2 = om * om;
    e.F = M.F0 + (1.0f - M.F0) * om2 * om2 * om;
    e.lam_o = smith_lambda(M.ndf, alpha, (float)e.cos_o, (float)(1.0 - e.cos_o * e.cos_o));
}

// Gate threshold of one grid node with n = w N 2^l trials (Eqs. 10, 16):
// P>=1 = 1 - (1 - p)^n from lp = log(1 - p), and the uniform (2k+1) 2^-24 is
// below P>=1  <=>  k < K.  Every branch is a select (the four nodes of a
// light are set up side by side): K = 0 when n <= 0 or p <= 0, P>=1 = 1 when
// p >= 1 (lp is then -inf or NaN and its value is discarded).
__device__ __forceinline__ uint32_t gate_K(float n, float p, float lp)
{
    const float pg = p >= 1.0f ? 1.0f : one_minus_exp(n * lp);
    const float kf = ceilf((pg * 16777216.0f - 1.0f) * 0.5f);
    const uint32_t K = kf >= 8388608.0f ? 8388608u : (kf > 0.0f ? (uint32_t)kf : 0u);
    return (n > 0.0f && p > 0.0f) ? K : 0u;
}

}  // namespace glint

namespace glint {
// d Lambda / d c and d Lambda / d alpha for direction cosine c (Smith, Eq. 2)
__device__ __forceinline__ void smith_lambda_grad(int ndf, float alpha, float c, float s2, float &dl_dc,
                                                  float &dl_da)
{
    if (s2 <= 0.0f) { dl_dc = 0.0f; dl_da = 0.0f; return; }
    const float a2 = alpha * alpha;
    const float T = s2 / (c * c);
    if (ndf == 0) {
        const float S = __builtin_amdgcn_sqrtf(1.0f + a2 * T);
        dl_dc = -a2 / (2.0f * c * c * c * S);
        dl_da = alpha * T / (2.0f * S);
    } else {
        const float a = 1.0f / (alpha * __builtin_amdgcn_sqrtf(T));
        const float dl_dacoef = -expf(-a * a) / (2.0f * a * a * 1.7724538509055160f);
        dl_dc = dl_dacoef / (alpha * s2 * __builtin_amdgcn_sqrtf(s2));
        dl_da = dl_dacoef * (-a / alpha);
    }
}

// the LDS record of a shaded pixel
__device__ __forceinline__ PixelRec make_rec(const Pixel &px, const Shared &sh)
{
    PixelRec r;
    const DevMaterial &M = sh.mats[px.mat];
    r.ex = (float)px.ex;
    r.ey = (float)px.ey;
    r.pk = (uint32_t)px.npr | ((uint32_t)px.n_nodes << 7) | ((uint32_t)px.mat << 10) |
           ((uint32_t)(px.level + 1024) << 15);
    r.alpha = px.alpha;
    // D_P = D(n) b / (R N P) with D(n) = 1/(pi alpha^2); L = E F G D_P / (4 <wi,n>)
    r.kpx = (float)(1.0 / ((double)M.R * (double)px.N * px.P * kPi * (double)px.alpha * (double)px.alpha * 4.0 *
                           px.cos_i));
    const float ci = (float)px.cos_i, si2 = (float)(1.0 - px.cos_i * px.cos_i);
    r.lam_i = smith_lambda(M.ndf, px.alpha, ci, si2);
    uint32_t d[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        d[g] = (uint32_t)(px.nl[g] - px.level) | ((uint32_t)px.nk[g] << 1) | ((uint32_t)px.nm[g] << 4);
        r.ng[g] = px.nw[g] * ldexpf(px.N, px.nl[g]);          // Eq. 10: w_g N 2^l_g trials
    }
    r.nd[0] = d[0] | (d[1] << 16);
    r.nd[1] = d[2] | (d[3] << 16);
    return r;
}

// Centre of sub-footprint kp of npr (Sec. 4.2: the distributed law over
// more areas): uniform along the major axis (ex, ey) = sigma0 e0 over length
// sigma0, centred on the pixel's uv.
__device__ __forceinline__ void probe_centre(double u, double v, double ex, double ey, int kp, int npr, double &cx,
                                             double &cy)
{
    const double off = ((double)kp + 0.5) * rcp_d((double)npr) - 0.5;
    cx = u + off * ex;
    cy = v + off * ey;
}

// Texel keys and barycentric weights of the simplex texels under a probe
// centred at (cx, cy) (Eq. 12, Sec. 6.2), for the four grid nodes whose key
// words (l + 1024) | k << 11 | m << 14 are w[g], under the material's hash
// root.  All four nodes are computed without branching (almost every pixel has
// four, and straight-line code lets the nodes' FP64 and hash chains
// interleave); the keys of nodes past the pixel's node count are never used.
// base[g] = H(root, w[g]), the node's key prefix (it depends on the pixel only)
__device__ __forceinline__ void texel_keys_from(double cx, double cy, const uint32_t w[4], const uint32_t base_g[4],
                                                const Shared &sh, uint32_t pre[4][3], float beta[4][3])
{
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int l = (int)(w[g] & 0x7ffu) - 1024, k = (w[g] >> 11) & 7, m = w[g] >> 14;
        int vi[3], vj[3];
        simplex_locate(cx, cy, l, k, m, sh, vi, vj, beta[g]);
        const uint32_t base = base_g[g];
        // vertex keys H(H(base, i), j): the triangle's vertices span two
        // columns i0 = vi[0] and i0 + 1 = vi[2], so two inner steps serve all three
        const uint32_t h0 = hstep(base, (uint32_t)vi[0]), h1 = hstep(base, (uint32_t)vi[2]);
        pre[g][0] = hstep(h0, (uint32_t)vj[0]);
        pre[g][1] = hstep(vi[1] == vi[0] ? h0 : h1, (uint32_t)vj[1]);
        pre[g][2] = hstep(h1, (uint32_t)vj[2]);
    }
}

__device__ __forceinline__ void texel_keys(double cx, double cy, const uint32_t w[4], uint32_t root, const Shared &sh,
                                           uint32_t pre[4][3], float beta[4][3])
{
    uint32_t base[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) base[g] = hstep(root, w[g]);
    texel_keys_from(cx, cy, w, base, sh, pre, beta);
}

// texel keys and barycentric weights of one probe's simplex texels (Sec. 6.2),
// staged in the caller's LDS columns ([node*3 + vertex][lane])
template <typename SM>
__device__ __forceinline__ void probe_texels(const PixelRec &R, double u, double v, int kp, const DevMaterial &M,
                                             const Shared &sh, uint32_t pre[4][3], SM &sm, uint32_t *key_sum)
{
    const int lane = threadIdx.x;
    const int npr = rec_npr(R), nn = rec_nodes(R);
    double cx, cy;
    probe_centre(u, v, (double)R.ex, (double)R.ey, kp, npr, cx, cy);
    uint32_t w[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) w[g] = rec_node_word(R, g);
    float beta[4][3];
    texel_keys(cx, cy, w, M.root, sh, pre, beta);
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            sm.pre[g * 3 + e][lane] = pre[g][e];
            sm.beta[g * 3 + e][lane] = beta[g][e];
            if (key_sum && g < nn) *key_sum += pre[g][e];
        }
}
}  // namespace glint
