/*
 * glint_oracle.c -- plain, slow, FP64 CPU reference of per-pixel glint shading
 * (Deliot & Belcour, "Real-Time Rendering of Glinty Appearances using
 * Distributed Binomial Laws on Anisotropic Grids", HPG 2023).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product library never does.  It
 * shares no code, header, table or constant generator with the HIP path.
 *
 * Every step follows the paper in its own order and notation, in FP64, from
 * the same FP32 inputs the GPU reads.  Where the paper leaves a choice open,
 * the reading taken is the one written next to the step.  Nothing here is
 * blocked, fused or reordered for speed.
 *
 *   step                                        paper passage
 *   footprint ellipse from screen derivatives   Sec. 5.1 (major/minor axes, rotation, ratio)
 *   probe split of over-long footprints         Sec. 4.2 (distribute over more than 2 areas)
 *   area level enclosure P_lo / P_hi            Sec. 5.2, Eq. 13; weights of Eq. 10
 *   ratio / orientation cell, pentagon          Sec. 5.2, Fig. 4; Sec. 6.1, Fig. 5
 *   prism -> tetrahedra split                   Sec. 6.1
 *   anisotropic grid transform                  Sec. 5.1, Eq. 12 (rotate then scale)
 *   simplex surface lattice                     Sec. 6.2, Fig. 6
 *   success probability p = R D(h)/D(n)         Sec. 3, Eq. 4
 *   tangent frame of the angular grid           Sec. 5.2, Eq. 14 (supplied tangent, else a basis of n)
 *   angular bilinear grid over projected h      Sec. 5.2, Eq. 14
 *   per-texel random numbers                    Sec. 3 (seeds on spatial / angular grids)
 *   gated Gaussian binomial                     Sec. 6.3, Eqs. 16-18
 *   uniforms from a precomputed table (variant) Sec. 6.3 (small texture of random numbers)
 *   distributed sum over grids                  Sec. 4.2, Eq. 10; Sec. 5.2
 *   glint NDF, BRDF, radiance                   Sec. 3, Eqs. 1-3
 *   baseline: Zirr-Kaplanyan counting (A/B)     Sec. 2, Eq. 7; Sec. 6.3, Eq. 15; Sec. 7
 *
 * Parity pins (tests that hold this file to the paper and to mathematics,
 * not to itself): footprint vs numpy SVD; NDF normalisation and Smith
 * masking integrals by quadrature; inverse normal CDF vs scipy; gated
 * binomial pmf vs its closed form through Phi; P(c=0) = (1-p)^n; area
 * conservation of the distributed weights; brute-force stratified flake
 * simulation for mean and variance of the distributed count; convergence
 * of the seed-averaged glint NDF to D(h); continuity across level, ratio,
 * orientation, lattice and angular-cell boundaries; the angular texels'
 * bilinear weights reconstructing the projected half vector, and the
 * distributed count as the bilinear blend of its values at the angular
 * texel centres (Eq. 14); frozen-branch finite differences
 * against free finite differences and against the forward-mode
 * (dual-number) derivatives of the same relaxed forward; the tangent frame orthonormal and
 * right-handed; the probe centres splitting the major axis into equal
 * segments; the Zirr-Kaplanyan baseline's branches against the binomial
 * and the floored-Gaussian closed forms, and its variance deficit; fmix32
 * to MurmurHash3's published test vectors.  The hash's key layout and
 * chaining and the angular cell size are definitions of this
 * implementation: parity unpinned beyond their statistical tests
 * (uniformity, independence) and the bit-exact match.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_PI 3.14159265358979323846
#define OG_MAX_NODES 4

/* ------------------------------------------------------------------ */
/* Public structures (mirrored by the ctypes wrapper in __init__.py).  */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t width, height;
    int64_t stride;
    const float *u, *v, *dudx, *dvdx, *dudy, *dvdy;
    const float *nx, *ny, *nz, *wx, *wy, *wz;
    const int32_t *material_id;   /* NULL: every pixel uses material 0 */
    const float *alpha_px;        /* NULL or per-pixel roughness */
    const float *log10_density_px;/* NULL or per-pixel log10 flake density */
    const float *tx, *ty, *tz;    /* NULL or per-pixel tangent (indexes the angular grid) */
} og_gbuffer;

typedef struct {
    int32_t ndf;                  /* 0 GGX, 1 Beckmann */
    float alpha, R, log10_density, micro_roughness, F0;
    uint32_t seed;
} og_material;

typedef struct { float dir[3]; float radiance[3]; } og_light;

/* rng_log2 = 0: gate uniforms hashed from their keys; 1..32: read from a
 * table of 2^rng_log2 words whose entry i is H(rng_seed, i) (Sec. 6.3, the
 * small precomputed texture of random numbers).
 * count_law 0: the distributed gated binomial (the method); 1: the counting
 * law of Zirr and Kaplanyan, an A/B baseline (see zk_count; integer counts,
 * so rounding must be 0). */
typedef struct { int32_t k_max, n_probe_max, rounding, rng_log2; uint32_t rng_seed; int32_t count_law; } og_params;

typedef struct {                  /* every plane is [height*stride] or NULL */
    uint32_t *flags;
    int32_t *n_probe, *level;
    uint32_t *cell, *key_sum, *akey_sum, *theta_sum, *count_sum, *n_open, *n_gate, *n_live;
    double *margin;               /* smallest margin of any decision (0: exactly on a boundary) */
    int32_t *margin_kind;
    double *margin_pos;           /* smallest margin rounding can decide (INFINITY when none) */
    int32_t *margin_pos_kind;
    double *b_light;              /* [n_light][height*stride]: raw distributed counts */
    uint32_t *lit;                /* bit l: some gate of light l opened in some probe (l < 32) */
    /* sampled per-texel dump (dump_slot NULL: none): dump_slot[height*stride]
     * is -1 or the slot in [0, dump_capacity) of the pixel; per slot, probe
     * k < dump_probes, node g < 4, lattice vertex e < 3, light l, angular
     * texel a < 4 (a & 1: x step, a >> 1: y step):
     *   dump_key  [cap][probes][4][3]       texel key
     *   dump_beta [cap][probes][4][3]       barycentric weight
     *   dump_theta[cap][probes][n_light][4][3][4]  slot-0 word of the texel
     *   dump_count[cap][probes][n_light][4][3][4]  count (0: gate closed)
     * every entry of a named slot is written (0 where there is no texel) */
    const int32_t *dump_slot;
    int32_t dump_capacity, dump_probes;
    uint32_t *dump_key;
    double *dump_beta;
    uint32_t *dump_theta;
    double *dump_count;
} og_debug;

/* flags */
#define OGF_SHADED      1u
#define OGF_CLAMP_RATIO 2u
#define OGF_CLAMP_P     4u
#define OGF_BAD_INPUT   8u
#define OGF_BACKFACING  16u
#define OGF_SKIPPED     32u
#define OGF_BAD_MAT     64u

/* margin kinds (which discrete decision came closest to its boundary) */
enum { MK_NONE = 0, MK_NPROBE, MK_RATIO, MK_ORIENT, MK_TRIANGLE, MK_TETRA,
       MK_LATTICE, MK_ANGULAR, MK_GATE, MK_COUNT, MK_LIGHT, MK_VIEW, MK_ZK_SWITCH,
       MK_PCLAMP, MK_TANGENT };

/* ------------------------------------------------------------------ */
/* Decision tape: records every light-dependent discrete decision of a */
/* pixel so that gradients can be taken with those branches frozen     */
/* (relaxed count, straight-through floor).                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t *buf;
    size_t len, cap, pos;
    int mode;                     /* 0 off, 1 record, 2 replay */
} og_tape;

static int32_t tape_dec(og_tape *T, int32_t computed)
{
    if (!T || T->mode == 0) return computed;
    if (T->mode == 1) {
        if (T->len == T->cap) {
            size_t nc = T->cap ? 2 * T->cap : 256;
            int32_t *nb = (int32_t *)realloc(T->buf, nc * sizeof(int32_t));
            if (!nb) abort();
            T->buf = nb; T->cap = nc;
        }
        T->buf[T->len++] = computed;
        return computed;
    }
    if (T->pos >= T->len) abort();
    return T->buf[T->pos++];
}

/* ------------------------------------------------------------------ */
/* Random numbers attached to grid texels (Sec. 3: seeds distributed   */
/* on a spatial and an angular grid).  The paper reads them from a     */
/* precomputed texture (Sec. 6.3); here they are an integer hash of    */
/* the texel key, with uint32 wraparound and no floating point.        */
/* Mixer: the MurmurHash3 32-bit finaliser (A. Appleby, public domain) */
/* ------------------------------------------------------------------ */
uint32_t og_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* one chaining step: absorb word w into state h */
uint32_t og_hash_step(uint32_t h, uint32_t w)
{
    return og_fmix32((h ^ w) + 0x9E3779B9u);
}

/* Entry i of the random-number table: H(seed, i).  The table is a pure
 * function of its index, so this oracle evaluates the entries it reads
 * instead of storing them. */
uint32_t og_rng_table_entry(uint32_t seed, uint32_t i)
{
    return og_hash_step(seed, i);
}

/* The 32-bit word behind the uniform of one gate or count: in hash mode
 * H(texel key, angular key); in table mode the table entry at the index
 * (texel key XOR angular key) mod 2^rng_log2.  With rng_log2 = 32 and
 * rng_seed = 0 both modes give the same word. */
static uint32_t gate_word(const og_params *prm, uint32_t pre, uint32_t ak)
{
    if (prm->rng_log2 == 0) return og_hash_step(pre, ak);
    uint32_t mask = prm->rng_log2 >= 32 ? 0xFFFFFFFFu : ((1u << prm->rng_log2) - 1u);
    return og_rng_table_entry(prm->rng_seed, (pre ^ ak) & mask);
}

/* key word of grid node (area level l, ratio level k, orientation m) */
static uint32_t node_word(int l, int k, int m)
{
    return (uint32_t)(l + 1024) | ((uint32_t)k << 11) | ((uint32_t)m << 14);
}

/* key word of angular texel (ai, aj) and random-number slot s in {0,1} */
static uint32_t angular_word(int ai, int aj, int s)
{
    return ((uint32_t)(ai + 16384) & 0x7FFFu) | (((uint32_t)(aj + 16384) & 0x7FFFu) << 15)
           | ((uint32_t)s << 30);
}

/* the full key chain of one random number: material seed, grid node
 * (l, k, m), simplex lattice vertex (i, j), angular texel (ai, aj), slot s */
uint32_t og_texel_hash(uint32_t seed, int l, int k, int m, int i, int j, int ai, int aj, int s)
{
    uint32_t s0 = og_hash_step(0x243F6A88u, seed);
    uint32_t base = og_hash_step(s0, node_word(l, k, m));
    uint32_t pre = og_hash_step(og_hash_step(base, (uint32_t)i), (uint32_t)j);
    uint32_t ak = og_hash_step(0x13198A2Eu, angular_word(ai, aj, s));
    return og_hash_step(pre, ak);
}

/* 23 random bits -> uniform strictly inside (0,1), exact in FP32 and FP64 */
static double uniform_of(uint32_t h)
{
    return (2.0 * (double)(h >> 9) + 1.0) * 0x1p-24;
}

/* ------------------------------------------------------------------ */
/* Standard normal inverse CDF, FP64.  Definition: the z with          */
/* Phi(z) = q, Phi(z) = erfc(-z/sqrt 2)/2.  Start from the Abramowitz  */
/* & Stegun 26.2.23 rational estimate (|err| < 4.5e-4) and refine with */
/* Halley steps on Phi(z) - q, using the lower tail for accuracy.      */
/* ------------------------------------------------------------------ */
double og_ndtri(double q)
{
    if (!(q > 0.0 && q < 1.0)) return q == 0.0 ? -INFINITY : (q == 1.0 ? INFINITY : NAN);
    if (q > 0.5) return -og_ndtri(1.0 - q);   /* 1-q exact for q in (0.5,1) */
    double t = sqrt(-2.0 * log(q));
    double z = -(t - (2.515517 + 0.802853 * t + 0.010328 * t * t) /
                      (1.0 + 1.432788 * t + 0.189269 * t * t + 0.001308 * t * t * t));
    for (int it = 0; it < 4; ++it) {
        double F = 0.5 * erfc(-z / sqrt(2.0));
        double f = exp(-0.5 * z * z) / sqrt(2.0 * OG_PI);
        double e = (F - q) / f;                    /* Newton step */
        z = z - e / (1.0 + 0.5 * z * e);           /* Halley correction */
    }
    return z;
}

/* ------------------------------------------------------------------ */
/* Microfacet pieces (Sec. 3, Eqs. 2-4).                               */
/* ------------------------------------------------------------------ */
/* NDF D(m) given cos(theta_m) = <n,m> */
double og_ndf(int ndf, double alpha, double cos_m)
{
    if (cos_m <= 0.0) return 0.0;
    double a2 = alpha * alpha, c2 = cos_m * cos_m;
    if (ndf == 0) {                                /* GGX / Trowbridge-Reitz */
        double d = c2 * (a2 - 1.0) + 1.0;
        return a2 / (OG_PI * d * d);
    } else {                                       /* Beckmann */
        double tan2 = (1.0 - c2) / c2;
        return exp(-tan2 / a2) / (OG_PI * a2 * c2 * c2);
    }
}

/* Smith Lambda for the same NDF, direction with cos(theta) = c */
double og_smith_lambda(int ndf, double alpha, double c)
{
    if (c >= 1.0) return 0.0;
    double tan2 = (1.0 - c * c) / (c * c);
    if (ndf == 0) return 0.5 * (-1.0 + sqrt(1.0 + alpha * alpha * tan2));
    double a = 1.0 / (alpha * sqrt(tan2));
    return 0.5 * (erf(a) - 1.0) + exp(-a * a) / (2.0 * a * sqrt(OG_PI));
}

static double smith_g1(int ndf, double alpha, double c)
{
    return 1.0 / (1.0 + og_smith_lambda(ndf, alpha, c));
}

/* Orthonormal basis around a unit normal: Duff et al., JCGT 6(1), 2017 */
static void onb(const double n[3], double t[3], double b[3])
{
    double sgn = copysign(1.0, n[2]);
    double a = -1.0 / (sgn + n[2]);
    double bb = n[0] * n[1] * a;
    t[0] = 1.0 + sgn * n[0] * n[0] * a; t[1] = sgn * bb; t[2] = -sgn * n[0];
    b[0] = bb; b[1] = sgn + n[1] * n[1] * a; b[2] = -n[1];
}

void og_onb(const double n[3], double t[3], double b[3]) { onb(n, t, b); }   /* for the pin tests */

static double dot3(const double a[3], const double b[3]) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

/* Tangent frame (t, b, n) whose first two axes index the angular grid
 * (Sec. 5.2, Eq. 14).  Reading: a supplied tangent is made orthogonal to the
 * unit normal (Gram-Schmidt) and normalised, and b = n x t (right-handed);
 * without one, the orthonormal basis of n above.  A supplied tangent within
 * about 1e-3 rad of n (sin^2 of their angle below 1e-6) defines no frame:
 * returns 0.  The margin of that decision is relative to the threshold. */
#define OG_TANGENT_MIN_SIN2 1e-6
static void upd_margin(double *mg, int *mk, double value, int kind);
static int tangent_frame(const double n[3], const double *tin, double t[3], double b[3],
                         double *mg, int *mk)
{
    if (!tin) { onb(n, t, b); return 1; }
    double tt = dot3(tin, tin);
    if (!(tt > 0.0)) return 0;
    double tn = dot3(tin, n);
    double tp[3] = {tin[0] - tn * n[0], tin[1] - tn * n[1], tin[2] - tn * n[2]};
    double s2 = dot3(tp, tp) / tt;                  /* sin^2 of the angle between t and n */
    if (mg) upd_margin(mg, mk, fabs(s2 - OG_TANGENT_MIN_SIN2) / OG_TANGENT_MIN_SIN2, MK_TANGENT);
    if (!(s2 >= OG_TANGENT_MIN_SIN2)) return 0;
    double l = sqrt(dot3(tp, tp));
    t[0] = tp[0] / l; t[1] = tp[1] / l; t[2] = tp[2] / l;
    b[0] = n[1] * t[2] - n[2] * t[1];
    b[1] = n[2] * t[0] - n[0] * t[2];
    b[2] = n[0] * t[1] - n[1] * t[0];
    return 1;
}

int og_tangent_frame(const double n[3], const double tin[3], double t[3], double b[3])
{
    return tangent_frame(n, tin, t, b, NULL, NULL);
}

/* Angular grid of Eq. 14: cells of size mr over the orthographic projection
 * (<h,t>, <h,b>) of the half vector, texel (i, j) centred at
 * ((i + 1/2) mr, (j + 1/2) mr).  Cell coordinates of h, measured from the
 * centre of texel (0, 0): */
static void angular_coords(const double h[3], const double t[3], const double b[3], double mr,
                           double *ax, double *ay)
{
    *ax = dot3(h, t) / mr - 0.5;
    *ay = dot3(h, b) / mr - 0.5;
}

/* bilinear weights of the four texels around (ax, ay), given the lower-left
 * texel (ai, aj): texel a is (ai + (a & 1), aj + (a >> 1)) and gets v[a] */
static void angular_weights(double ax, double ay, int ai, int aj, double v[4])
{
    double fx = ax - ai, fy = ay - aj;
    v[0] = (1.0 - fx) * (1.0 - fy);
    v[1] = fx * (1.0 - fy);
    v[2] = (1.0 - fx) * fy;
    v[3] = fx * fy;
}

/* the four angular texels of h and their weights (for the pin tests) */
void og_angular_texels(const double h[3], const double t[3], const double b[3], double mr,
                       int *ai, int *aj, double v[4])
{
    double ax, ay;
    angular_coords(h, t, b, mr, &ax, &ay);
    *ai = (int)floor(ax);
    *aj = (int)floor(ay);
    angular_weights(ax, ay, *ai, *aj, v);
}

/* centre of sub-footprint kp of n_pr (Sec. 4.2, reading S25): uniform along
 * the major axis (angle phi) over the major-axis length sigma0 */
static void probe_centre(double u, double v, double phi, double sigma0, int n_pr, int kp, double *cx, double *cy)
{
    double off = ((kp + 0.5) / n_pr - 0.5) * sigma0;
    *cx = u + off * cos(phi);
    *cy = v + off * sin(phi);
}

void og_probe_centre(double u, double v, double phi, double sigma0, int n_pr, int kp, double *cx, double *cy)
{
    probe_centre(u, v, phi, sigma0, n_pr, kp, cx, cy);
}

static int normalize3(double a[3])
{
    double l = sqrt(dot3(a, a));
    if (!(l > 0.0) || !isfinite(l)) return 0;
    a[0] /= l; a[1] /= l; a[2] /= l;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Footprint (Sec. 5.1): ellipse of the pixel's image under the UV     */
/* Jacobian J = [du/dx du/dy; dv/dx dv/dy].  Axes are the singular     */
/* vectors of J; the area is |det J|; the rotation is the major axis   */
/* angle taken mod pi; the ratio is sigma0/sigma1.                     */
/* ------------------------------------------------------------------ */
int og_footprint(double dudx, double dvdx, double dudy, double dvdy,
                 double *P, double *r, double *phi, double *sigma0)
{
    double a = dudx * dudx + dudy * dudy;          /* J J^T */
    double b = dudx * dvdx + dudy * dvdy;
    double c = dvdx * dvdx + dvdy * dvdy;
    double det = dudx * dvdy - dudy * dvdx;
    *P = fabs(det);
    if (!(*P > 0.0) || !isfinite(*P)) return 0;
    double hm = 0.5 * (a + c), hd = 0.5 * (a - c);
    double s0sq = hm + sqrt(hd * hd + b * b);      /* larger eigenvalue */
    double rr = s0sq / *P;                         /* sigma0/sigma1 = sigma0^2/|det| */
    *r = rr < 1.0 ? 1.0 : rr;
    double ph = 0.5 * atan2(2.0 * b, a - c);
    if (ph < 0.0) ph += OG_PI;
    *phi = ph;
    *sigma0 = sqrt(s0sq);
    return 1;
}

/* ------------------------------------------------------------------ */
/* Grid nodes of the anisotropic family enclosing a sub-footprint of   */
/* area Pk, ratio rk, orientation phi (Sec. 5.2 + Sec. 6.1).           */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;                         /* number of tetrahedron vertices (<= 4) */
    int l[OG_MAX_NODES], k[OG_MAX_NODES], m[OG_MAX_NODES];
    double w[OG_MAX_NODES];
    int level, kappa, j, tri, pivot, D;
} og_nodes;

/* Decisions whose value is an exact function of exactly representable
 * inputs wherever it lands on its boundary (probe count, ratio level,
 * orientation, triangle, tetrahedron): an exact tie is reproduced by any
 * implementation that rounds its operations correctly.  The others (lattice,
 * angular cell, gate, count, light and view validity) follow rounded chains
 * (products, square roots, trigonometry) that implementations may round
 * differently, so an exact tie there is as undecidable as a near one. */
static int tie_exact(int kind)
{
    return kind == MK_NPROBE || kind == MK_RATIO || kind == MK_ORIENT || kind == MK_TRIANGLE || kind == MK_TETRA;
}

/* margins of a pixel's decisions: mg[0] / mk[0] the smallest of all, mg[1] /
 * mk[1] the smallest one that rounding can decide differently (positive, or
 * an exact tie of a rounded decision).  A zero elsewhere in the pixel must
 * not hide it. */
static void upd_margin(double *mg, int *mk, double value, int kind)
{
    if (value < mg[0]) { mg[0] = value; mk[0] = kind; }
    if ((value > 0.0 || !tie_exact(kind)) && value < mg[1]) { mg[1] = value; mk[1] = kind; }
}

/* distance of x to the nearest integer in [lo, hi] */
static double dist_int(double x, double lo, double hi)
{
    double k = floor(x + 0.5);
    if (k < lo) k = lo;
    if (k > hi) k = hi;
    return fabs(x - k);
}

void og_grid_nodes(double Pk, double rk, double phi, int K, og_nodes *out,
                   double *mg, int *mk)
{
    /* area levels: P_lo = 2^floor(log2 P), P_hi = 2^ceil(log2 P) (Eq. 13);
     * the weight of the top level is (P - P_lo)/(P_hi - P_lo) (Eq. 10). */
    int ex;
    double fr = frexp(Pk, &ex);                    /* Pk = fr 2^ex, fr in [0.5,1) */
    int l = ex - 1;
    double ts = 2.0 * fr - 1.0;                    /* (Pk - 2^l) / 2^l in [0,1) */
    out->level = l;

    /* ratio / orientation cell and barycentric weights over its nodes */
    int nk[3], nm[3];
    double lam[3];
    int nv;
    if (K == 0) {                                   /* isotropic family only */
        nv = 1; nk[0] = 0; nm[0] = 0; lam[0] = 1.0;
        out->kappa = 0; out->j = 0; out->tri = 0;
    } else {
        double rho = log2(rk);                      /* circle k <-> r = 2^k */
        if (rho < 0.0) rho = 0.0;
        if (rho > K) rho = K;
        int kap = (int)floor(rho);
        if (kap > K - 1) kap = K - 1;
        upd_margin(mg, mk, dist_int(rho, 1.0, K - 1.0), MK_RATIO);
        double u = rho - kap;
        int M = 1 << (kap + 1);                     /* orientations on ring kap over [0,pi) */
        double q = phi / (OG_PI / M);
        int j = (int)floor(q);
        if (j < 0) j = 0;
        if (j > M - 1) j = M - 1;
        upd_margin(mg, mk, dist_int(q, 0.0, (double)M), MK_ORIENT);
        double t = q - j;
        int Mo = 2 * M;                              /* outer ring has twice as many */
        /* pentagon (u,t): I0=(0,0) I1=(0,1) O0=(1,0) O1=(1,1/2) O2=(1,1) */
        int I0k = kap, I0m = j, I1k = kap, I1m = (j + 1) % M;
        int O0k = kap + 1, O0m = 2 * j, O1k = kap + 1, O1m = 2 * j + 1, O2k = kap + 1, O2m = (2 * j + 2) % Mo;
        upd_margin(mg, mk, fabs(t - 0.5 * u), MK_TRIANGLE);
        upd_margin(mg, mk, fabs(t - (1.0 - 0.5 * u)), MK_TRIANGLE);
        if (t <= 0.5 * u) {                          /* T1 = (I0, O0, O1) */
            out->tri = 0;
            nk[0] = I0k; nm[0] = I0m; lam[0] = 1.0 - u;
            nk[1] = O0k; nm[1] = O0m; lam[1] = u - 2.0 * t;
            nk[2] = O1k; nm[2] = O1m; lam[2] = 2.0 * t;
        } else if (t >= 1.0 - 0.5 * u) {             /* T3 = (I1, O2, O1) */
            out->tri = 2;
            nk[0] = I1k; nm[0] = I1m; lam[0] = 1.0 - u;
            nk[1] = O2k; nm[1] = O2m; lam[1] = u - 2.0 * (1.0 - t);
            nk[2] = O1k; nm[2] = O1m; lam[2] = 2.0 * (1.0 - t);
        } else {                                     /* T2 = (I0, I1, O1) */
            out->tri = 1;
            nk[0] = I0k; nm[0] = I0m; lam[0] = 1.0 - t - 0.5 * u;
            nk[1] = I1k; nm[1] = I1m; lam[1] = t - 0.5 * u;
            nk[2] = O1k; nm[2] = O1m; lam[2] = u;
        }
        for (int a = 0; a < 3; ++a) {
            if (lam[a] < 0.0) lam[a] = 0.0;
            if (nk[a] == 0) nm[a] = 0;               /* every ring-0 node is the isotropic grid */
        }
        nv = 3;
        out->kappa = kap; out->j = j;
    }

    /* merge coincident nodes, then sort by global key (k, m) ascending */
    int dk[3], dm[3];
    double dl[3];
    int D = 0;
    for (int a = 0; a < nv; ++a) {
        int found = -1;
        for (int b = 0; b < D; ++b)
            if (dk[b] == nk[a] && dm[b] == nm[a]) found = b;
        if (found >= 0) dl[found] += lam[a];
        else { dk[D] = nk[a]; dm[D] = nm[a]; dl[D] = lam[a]; ++D; }
    }
    for (int a = 1; a < D; ++a)                      /* insertion sort */
        for (int b = a; b > 0 && (dk[b - 1] * 64 + dm[b - 1]) > (dk[b] * 64 + dm[b]); --b) {
            int tk = dk[b]; dk[b] = dk[b - 1]; dk[b - 1] = tk;
            int tm = dm[b]; dm[b] = dm[b - 1]; dm[b - 1] = tm;
            double tl = dl[b]; dl[b] = dl[b - 1]; dl[b - 1] = tl;
        }

    /* prism (triangle x scale) -> tetrahedron: move the top-level mass ts
     * onto the nodes from the highest key down.  The three tetrahedra this
     * selects tile the prism and agree on shared faces (split by key order). */
    double top[3] = {0, 0, 0};
    double rem = ts;
    int pivot = 0;
    for (int a = D - 1; a >= 0; --a) {
        if (a > 0) upd_margin(mg, mk, fabs(rem - dl[a]), MK_TETRA);
        if (rem <= dl[a] || a == 0) {
            top[a] = rem < dl[a] ? rem : dl[a];
            pivot = a;
            break;
        }
        top[a] = dl[a];
        rem -= dl[a];
    }
    int n = 0;
    for (int a = 0; a <= pivot; ++a) {               /* bottom level l */
        out->l[n] = l; out->k[n] = dk[a]; out->m[n] = dm[a];
        out->w[n] = dl[a] - top[a];
        ++n;
    }
    for (int a = pivot; a < D; ++a) {                /* top level l+1 */
        out->l[n] = l + 1; out->k[n] = dk[a]; out->m[n] = dm[a];
        out->w[n] = top[a];
        ++n;
    }
    out->n = n;
    out->pivot = pivot;
    out->D = D;
}

/* ------------------------------------------------------------------ */
/* Simplex lattice of one grid node (Sec. 5.1 Eq. 12 + Sec. 6.2):      */
/* rotate the point by -phi_g, scale to cells of area A = 2^l and      */
/* aspect r = 2^k, skew to the triangular lattice and locate the       */
/* triangle.  Returns three lattice vertices and barycentric weights.  */
/* ------------------------------------------------------------------ */
void og_simplex(double cx, double cy, int l, int k, int m,
                int vi[3], int vj[3], double beta[3], double *mg, int *mk)
{
    double phig = (k == 0) ? 0.0 : (double)m * OG_PI / (double)(1 << (k + 1));
    double cph = cos(phig), sph = sin(phig);
    double qx = cph * cx + sph * cy;
    double qy = -sph * cx + cph * cy;
    double wx = sqrt(ldexp(1.0, l + k));           /* cell side along the major axis */
    double wy = sqrt(ldexp(1.0, l - k));           /* cell side along the minor axis */
    double x = qx / wx, y = qy / wy;
    double Lx = x + 0.5 * y, Ly = y;               /* skew: triangular lattice -> integer lattice */
    double fi = floor(Lx), fj = floor(Ly);
    double f = Lx - fi, g = Ly - fj;
    int i = (int)fi, j = (int)fj;
    upd_margin(mg, mk, fabs(Lx - floor(Lx + 0.5)), MK_LATTICE);
    upd_margin(mg, mk, fabs(Ly - floor(Ly + 0.5)), MK_LATTICE);
    upd_margin(mg, mk, fabs(f - g), MK_LATTICE);
    if (f >= g) {
        vi[0] = i; vj[0] = j; vi[1] = i + 1; vj[1] = j; vi[2] = i + 1; vj[2] = j + 1;
        beta[0] = 1.0 - f; beta[1] = f - g; beta[2] = g;
    } else {
        vi[0] = i; vj[0] = j; vi[1] = i; vj[1] = j + 1; vi[2] = i + 1; vj[2] = j + 1;
        beta[0] = 1.0 - g; beta[1] = g - f; beta[2] = f;
    }
}

/* ------------------------------------------------------------------ */
/* Gated Gaussian binomial (Sec. 6.3, Eqs. 16-18).  Success of the     */
/* gate is theta0 < P>=1 (the paper's trials succeed when X < p).      */
/* rounding 0: c = max(1, floor(1 + mu + sigma Phi^-1(theta1)));       */
/* rounding 1 (relaxed): c = max(1, 1 + mu + sigma Phi^-1(theta1)).    */
/* ------------------------------------------------------------------ */
double og_gated_count(double n, double p, double theta0, double theta1, int rounding)
{
    double pg;
    if (!(n > 0.0) || !(p > 0.0)) pg = 0.0;
    else if (p >= 1.0) pg = 1.0;
    else pg = -expm1(n * log1p(-p));
    if (!(theta0 < pg)) return 0.0;
    double mm = n - 1.0 > 0.0 ? n - 1.0 : 0.0;
    double mu = mm * p, sigma = sqrt(mm * p * (1.0 - p));
    double x = 1.0 + mu + sigma * og_ndtri(theta1);
    if (rounding == 0) x = floor(x);
    return x > 1.0 ? x : 1.0;
}

/* ------------------------------------------------------------------ */
/* Counting law of Zirr and Kaplanyan, the prior art the method        */
/* replaces (Sec. 2, Eq. 7; Sec. 6.3, Eq. 15), kept as an A/B baseline. */
/* Every grid node counts the flakes of its whole cell, n = N A_g      */
/* trials, and the node outputs are mixed with the interpolation       */
/* weights w_g (Eq. 7: a linear mix of binomial outputs, here over the */
/* nodes of the grid family instead of two LOD levels).  One count:    */
/*   n p > 5, or n above the Bernoulli loop limit 16 (Sec. 7):          */
/*       c = max(0, floor(n p + sqrt(n p (1-p)) Phi^-1(theta_0)))       */
/*   otherwise t = floor(n + 1/2) Bernoulli trials:                     */
/*       c = #{k = 1..t : theta_k < p},  theta_k the uniform of H(h0, k) */
/* with h0 the texel's slot-0 word and theta_0 its uniform; a trial     */
/* succeeds when theta < p, as the gates do (the paper's X_i < p).      */
/* *gauss: 1 on the Gaussian branch; *trials: Bernoulli trials drawn.   */
/* ------------------------------------------------------------------ */
#define OG_ZK_LOOP_MAX 16.0
static double zk_count(double n, double p, uint32_t h0, double *mg, int *mk, int *gauss, int *trials)
{
    const double mu = n * p;
    upd_margin(mg, mk, fabs(mu - 5.0) / 5.0, MK_ZK_SWITCH);
    upd_margin(mg, mk, fabs(n - OG_ZK_LOOP_MAX) / OG_ZK_LOOP_MAX, MK_ZK_SWITCH);
    if (mu > 5.0 || n > OG_ZK_LOOP_MAX) {
        *gauss = 1;
        *trials = 0;
        const double sd = sqrt(mu * (1.0 - p));
        const double z = og_ndtri(uniform_of(h0));
        const double x = mu + sd * z;
        if (x >= 0.5)   /* floor(x) decides the count; its error scale is mu + sd |z| */
            upd_margin(mg, mk, fabs(x - floor(x + 0.5)) / (mu + sd * fabs(z) + 1.0), MK_COUNT);
        const double c = floor(x);
        return c > 0.0 ? c : 0.0;
    }
    *gauss = 0;
    upd_margin(mg, mk, fabs(n + 0.5 - floor(n + 1.0)) / (n > 1.0 ? n : 1.0), MK_ZK_SWITCH);
    const int t = (int)floor(n + 0.5);
    *trials = t;
    double c = 0.0;
    for (int k = 1; k <= t; ++k) {
        const double th = uniform_of(og_hash_step(h0, (uint32_t)k));
        upd_margin(mg, mk, fabs(th - p) / (p > 0x1p-24 ? p : 0x1p-24), MK_GATE);
        if (th < p) c += 1.0;
    }
    return c;
}

double og_zk_count(double n, double p, uint32_t h0, int *gauss, int *trials)
{
    double mg[2] = {INFINITY, INFINITY};
    int mk[2] = {MK_NONE, MK_NONE};
    return zk_count(n, p, h0, mg, mk, gauss, trials);
}

/* ------------------------------------------------------------------ */
/* One pixel.                                                          */
/* ------------------------------------------------------------------ */
typedef struct {
    double u, v, dudx, dvdx, dudy, dvdy, n[3], wi[3];
    int mat;
    double alpha, log10N;          /* effective values (material or per-pixel) */
    int has_t;                     /* a tangent t[] was supplied */
    double t[3];
} og_px_in;

typedef struct {
    double alpha_shift;            /* added to the pixel's alpha (gradients) */
    double lnN_shift;              /* added to ln N */
    const double *dirs;            /* [n_light][3] raw light directions (perturbable) */
} og_perturb;

typedef struct {
    double rgb[3];
    uint32_t flags, cell, key_sum, akey_sum, theta_sum, count_sum, n_open, n_gate, n_live, lit;
    int32_t n_probe, level;
    double margin[2];              /* smallest, smallest positive (see upd_margin) */
    int32_t margin_kind[2];
    double b[64];                  /* raw distributed count per light (first 64 lights) */
} og_px_out;

/* one pixel's slot of the per-texel dump (zero-filled by the caller) */
typedef struct {
    int probes;
    uint32_t *key;                /* [probes][4][3] */
    double *beta;
    uint32_t *theta;              /* [probes][n_light][4][3][4] */
    double *count;
} og_dump;

static void shade_pixel(const og_px_in *in, const og_material *mat, const og_light *lights,
                        int n_light, const og_params *prm, const og_perturb *pt,
                        og_tape *T, og_px_out *o, const og_dump *dd)
{
    memset(o, 0, sizeof(*o));
    o->margin[0] = o->margin[1] = INFINITY;
    o->margin_kind[0] = o->margin_kind[1] = MK_NONE;
    double *mg = o->margin;
    int *mk = o->margin_kind;

    const int K = prm->k_max;
    const double alpha = in->alpha + (pt ? pt->alpha_shift : 0.0);
    const double lnN = in->log10N * log(10.0) + (pt ? pt->lnN_shift : 0.0);
    const double N = exp(lnN);                      /* flakes per unit UV area */
    const double R = mat->R;

    double nrm[3] = {in->n[0], in->n[1], in->n[2]};
    double wi[3] = {in->wi[0], in->wi[1], in->wi[2]};
    if (!normalize3(nrm) || !normalize3(wi)) { o->flags |= OGF_BAD_INPUT; return; }
    /* the frame of the angular grid (Eq. 14) */
    double tt[3], bb[3];
    if (!tangent_frame(nrm, in->has_t ? in->t : NULL, tt, bb, mg, mk)) { o->flags |= OGF_BAD_INPUT; return; }

    double P, r, phi, sigma0;
    if (!og_footprint(in->dudx, in->dvdx, in->dudy, in->dvdy, &P, &r, &phi, &sigma0)) {
        o->flags |= OGF_BAD_INPUT;
        return;
    }
    double cos_i = dot3(nrm, wi);
    upd_margin(mg, mk, fabs(cos_i), MK_VIEW);
    if (!(cos_i > 0.0)) { o->flags |= OGF_BACKFACING; return; }

    /* footprints longer than the family's largest ratio are distributed
     * over n_pr equal sub-footprints along the major axis (Sec. 4.2) */
    double qn = r / ldexp(1.0, K);
    int n_pr = (int)ceil(qn);
    if (n_pr < 1) n_pr = 1;
    if (n_pr > prm->n_probe_max) n_pr = prm->n_probe_max;
    upd_margin(mg, mk, dist_int(qn, 1.0, (double)prm->n_probe_max) / (qn > 1.0 ? qn : 1.0), MK_NPROBE);
    double Pk = P / n_pr;
    double rk = r / n_pr;
    if (rk > ldexp(1.0, K)) { rk = ldexp(1.0, K); o->flags |= OGF_CLAMP_RATIO; }
    o->n_probe = n_pr;

    og_nodes nodes;
    og_grid_nodes(Pk, rk, phi, K, &nodes, mg, mk);
    o->level = nodes.level;
    o->cell = (uint32_t)nodes.kappa | ((uint32_t)nodes.j << 3) | ((uint32_t)nodes.tri << 9)
              | ((uint32_t)nodes.pivot << 11) | ((uint32_t)nodes.D << 13) | ((uint32_t)nodes.n << 15);

    /* per-light quantities that do not depend on the probe */
    const double mr = mat->micro_roughness;
    const double Dn = 1.0 / (OG_PI * alpha * alpha);  /* D(n) for GGX and Beckmann */
    const uint32_t s0 = og_hash_step(0x243F6A88u, mat->seed);

    int lv[64], ai[64], aj[64];
    double vw[64][4], pl[64], Fl[64], Gl[64];
    uint32_t akey[64][4][2];
    int NL = n_light < 64 ? n_light : 64;
    for (int li = 0; li < NL; ++li) {
        double wo[3];
        if (pt && pt->dirs) { wo[0] = pt->dirs[3*li]; wo[1] = pt->dirs[3*li+1]; wo[2] = pt->dirs[3*li+2]; }
        else { wo[0] = lights[li].dir[0]; wo[1] = lights[li].dir[1]; wo[2] = lights[li].dir[2]; }
        int ok = normalize3(wo);
        double cos_o = ok ? dot3(nrm, wo) : -1.0;
        double h[3] = {wi[0] + wo[0], wi[1] + wo[1], wi[2] + wo[2]};
        ok = ok && (cos_o > 0.0) && normalize3(h);
        if (ok) upd_margin(mg, mk, fabs(cos_o), MK_LIGHT);
        lv[li] = tape_dec(T, ok);
        if (!lv[li]) continue;
        double cos_h = dot3(nrm, h);
        /* Eq. 4: p = R D(h)/D(n), clamped to a probability */
        double praw = R * og_ndf(mat->ndf, alpha, cos_h) / Dn;
        upd_margin(mg, mk, fabs(praw - 1.0), MK_PCLAMP);
        int pc = tape_dec(T, praw > 1.0);
        if (pc) o->flags |= OGF_CLAMP_P;
        pl[li] = pc ? 1.0 : praw;
        /* Eq. 14: bilinear over the 4 nearest texels of the angular grid,
         * indexed by the orthographic projection of h, cell size mr */
        double ax, ay;
        angular_coords(h, tt, bb, mr, &ax, &ay);
        upd_margin(mg, mk, fabs(ax - floor(ax + 0.5)), MK_ANGULAR);
        upd_margin(mg, mk, fabs(ay - floor(ay + 0.5)), MK_ANGULAR);
        ai[li] = tape_dec(T, (int32_t)floor(ax));
        aj[li] = tape_dec(T, (int32_t)floor(ay));
        angular_weights(ax, ay, ai[li], aj[li], vw[li]);
        for (int a = 0; a < 4; ++a)
            for (int s = 0; s < 2; ++s) {
                akey[li][a][s] = og_hash_step(0x13198A2Eu, angular_word(ai[li] + (a & 1), aj[li] + (a >> 1), s));
            }
        for (int a = 0; a < 4; ++a) o->akey_sum += akey[li][a][0];
        /* Schlick Fresnel and separable Smith masking (Eq. 2) */
        double ch = dot3(wi, h);
        double F0 = mat->F0;
        double om = 1.0 - ch;
        Fl[li] = F0 + (1.0 - F0) * om * om * om * om * om;
        Gl[li] = smith_g1(mat->ndf, alpha, cos_i) * smith_g1(mat->ndf, alpha, cos_o);
    }

    double bsum[64];
    for (int li = 0; li < NL; ++li) bsum[li] = 0.0;

    for (int kp = 0; kp < n_pr; ++kp) {
        double cx, cy;
        probe_centre(in->u, in->v, phi, sigma0, n_pr, kp, &cx, &cy);
        int vi[OG_MAX_NODES][3], vj[OG_MAX_NODES][3];
        double beta[OG_MAX_NODES][3];
        uint32_t pre[OG_MAX_NODES][3];
        /* this probe's part of the per-texel dump, or NULL */
        const int dump = dd && kp < dd->probes;
        uint32_t *dk = dump ? dd->key + (size_t)kp * 12 : NULL;
        double *db = dump ? dd->beta + (size_t)kp * 12 : NULL;
        for (int g = 0; g < nodes.n; ++g) {
            og_simplex(cx, cy, nodes.l[g], nodes.k[g], nodes.m[g], vi[g], vj[g], beta[g], mg, mk);
            uint32_t base = og_hash_step(s0, node_word(nodes.l[g], nodes.k[g], nodes.m[g]));
            for (int e = 0; e < 3; ++e) {
                pre[g][e] = og_hash_step(og_hash_step(base, (uint32_t)vi[g][e]), (uint32_t)vj[g][e]);
                o->key_sum += pre[g][e];
                if (dump) { dk[g * 3 + e] = pre[g][e]; db[g * 3 + e] = beta[g][e]; }
            }
        }
        for (int li = 0; li < NL; ++li) {
            if (!lv[li]) continue;
            double p = pl[li];
            uint32_t *dt = dump ? dd->theta + ((size_t)kp * n_light + li) * 48 : NULL;
            double *dc = dump ? dd->count + ((size_t)kp * n_light + li) * 48 : NULL;
            for (int g = 0; g < nodes.n; ++g) {
                if (prm->count_law == 1) {
                    /* Eq. 7 baseline: node g counts its whole cell (N A_g
                     * trials) and its output enters with weight w_g */
                    const double nz = N * ldexp(1.0, nodes.l[g]);
                    for (int e = 0; e < 3; ++e)
                        for (int a = 0; a < 4; ++a) {
                            uint32_t h0 = gate_word(prm, pre[g][e], akey[li][a][0]);
                            o->theta_sum += h0;
                            o->n_gate++;
                            int gauss, trials;
                            double c = zk_count(nz, p, h0, mg, mk, &gauss, &trials);
                            if (dump) { dt[g * 12 + e * 4 + a] = h0; dc[g * 12 + e * 4 + a] = c; }
                            o->n_open += (uint32_t)gauss;
                            o->n_live += (uint32_t)trials;
                            o->count_sum += (uint32_t)c;
                            if (c > 0.0 && li < 32) o->lit |= 1u << li;
                            bsum[li] += nodes.w[g] * beta[g][e] * vw[li][a] * c;
                        }
                    continue;
                }
                /* Eq. 10: node g receives w_g N A_g trials */
                double ng = nodes.w[g] * N * ldexp(1.0, nodes.l[g]);
                double pg;
                if (!(ng > 0.0) || !(p > 0.0)) pg = 0.0;
                else if (p >= 1.0) pg = 1.0;
                else pg = -expm1(ng * log1p(-p));    /* Eq. 16 */
                double mm = ng - 1.0 > 0.0 ? ng - 1.0 : 0.0;
                double mu = mm * p;                   /* Eq. 17 */
                double sg = sqrt(mm * p * (1.0 - p));
                int live = pg > 0x1p-24;
                for (int e = 0; e < 3; ++e)
                    for (int a = 0; a < 4; ++a) {
                        uint32_t h0 = gate_word(prm, pre[g][e], akey[li][a][0]);
                        double th0 = uniform_of(h0);
                        o->theta_sum += h0;
                        o->n_gate++;
                        if (live) {
                            o->n_live++;
                            upd_margin(mg, mk, fabs(th0 - pg) / (pg > 0x1p-24 ? pg : 0x1p-24), MK_GATE);
                        }
                        int open = tape_dec(T, th0 < pg);
                        double c = 0.0;
                        if (open) {                   /* Eq. 18 with the gate read as theta0 < P>=1 */
                            o->n_open++;
                            if (li < 32) o->lit |= 1u << li;
                            uint32_t h1 = gate_word(prm, pre[g][e], akey[li][a][1]);
                            double x = 1.0 + mu + sg * og_ndtri(uniform_of(h1));
                            if (x >= 1.5) {
                                double k = floor(x + 0.5);
                                upd_margin(mg, mk, fabs(x - k) / (x > 1.0 ? x : 1.0), MK_COUNT);
                            }
                            if (prm->rounding == 0) {
                                double xf = floor(x);
                                c = xf > 1.0 ? xf : 1.0;
                                o->count_sum += (uint32_t)c;
                            } else {
                                int br = tape_dec(T, x >= 1.0);
                                c = br ? x : 1.0;
                            }
                        }
                        if (dump) { dt[g * 12 + e * 4 + a] = h0; dc[g * 12 + e * 4 + a] = c; }
                        bsum[li] += beta[g][e] * vw[li][a] * c;
                    }
            }
        }
    }

    /* Eqs. 1-4: D_P = D(n) b / (R N P); L = sum_l E_l F G D_P / (4 <wi,n>) */
    for (int li = 0; li < NL; ++li) {
        o->b[li] = bsum[li];
        if (!lv[li]) continue;
        double DP = Dn * bsum[li] / (R * N * P);
        double f = Fl[li] * Gl[li] * DP / (4.0 * cos_i);
        for (int ch = 0; ch < 3; ++ch) o->rgb[ch] += (double)lights[li].radiance[ch] * f;
    }
    o->flags |= OGF_SHADED;
}

static int load_pixel(const og_gbuffer *gb, const og_material *mats, int n_mat, int64_t idx,
                      og_px_in *in, uint32_t *flags)
{
    int mat = gb->material_id ? gb->material_id[idx] : 0;
    if (mat < 0) { *flags = OGF_SKIPPED; return 0; }
    if (mat >= n_mat) { *flags = OGF_BAD_MAT; return 0; }
    in->mat = mat;
    in->u = gb->u[idx]; in->v = gb->v[idx];
    in->dudx = gb->dudx[idx]; in->dvdx = gb->dvdx[idx];
    in->dudy = gb->dudy[idx]; in->dvdy = gb->dvdy[idx];
    in->n[0] = gb->nx[idx]; in->n[1] = gb->ny[idx]; in->n[2] = gb->nz[idx];
    in->wi[0] = gb->wx[idx]; in->wi[1] = gb->wy[idx]; in->wi[2] = gb->wz[idx];
    in->alpha = gb->alpha_px ? (double)gb->alpha_px[idx] : (double)mats[mat].alpha;
    in->log10N = gb->log10_density_px ? (double)gb->log10_density_px[idx] : (double)mats[mat].log10_density;
    in->has_t = gb->tx != NULL;
    in->t[0] = in->has_t ? gb->tx[idx] : 0.0;
    in->t[1] = in->has_t ? gb->ty[idx] : 0.0;
    in->t[2] = in->has_t ? gb->tz[idx] : 0.0;
    double vals[17] = {in->u, in->v, in->dudx, in->dvdx, in->dudy, in->dvdy, in->n[0], in->n[1],
                       in->n[2], in->wi[0], in->wi[1], in->wi[2], in->alpha, in->log10N,
                       in->t[0], in->t[1], in->t[2]};
    for (int i = 0; i < 17; ++i)
        if (!isfinite(vals[i])) { *flags = OGF_BAD_INPUT; return 0; }
    if (!(in->alpha > 0.0)) { *flags = OGF_BAD_INPUT; return 0; }
    return 1;
}

static void set_threads(int n_threads)
{
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
}

/* Forward shading of rows [row0, row1).  out_rgb: [3][height*stride]. */
int og_shade(const og_gbuffer *gb, const og_material *mats, int n_mat, const og_light *lights,
             int n_light, const og_params *prm, double *out_rgb, og_debug *dbg,
             int row0, int row1, int n_threads)
{
    if (!gb || !mats || n_mat <= 0 || n_light < 0 || n_light > 64 || !prm || !out_rgb) return -1;
    if (prm->k_max < 0 || prm->k_max > 4 || prm->n_probe_max < 1) return -1;
    if (prm->rng_log2 < 0 || prm->rng_log2 > 32) return -1;
    if (prm->count_law != 0 && !(prm->count_law == 1 && prm->rounding == 0)) return -1;
    if (gb->tx && (!gb->ty || !gb->tz)) return -1;
    if (dbg && dbg->dump_slot &&
        (!dbg->dump_key || !dbg->dump_beta || !dbg->dump_theta || !dbg->dump_count ||
         dbg->dump_capacity < 1 || dbg->dump_probes < 1))
        return -1;
    if (row0 < 0) row0 = 0;
    if (row1 > gb->height) row1 = gb->height;
    const int64_t npx = (int64_t)gb->height * gb->stride;
    set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = row0; y < row1; ++y) {
        for (int x = 0; x < gb->width; ++x) {
            int64_t idx = (int64_t)y * gb->stride + x;
            og_px_in in;
            og_px_out o;
            uint32_t lflags = 0;
            og_dump dslot, *dd = NULL;
            const int32_t slot = (dbg && dbg->dump_slot) ? dbg->dump_slot[idx] : -1;
            if (slot >= 0 && slot < dbg->dump_capacity) {
                const size_t P = (size_t)dbg->dump_probes, ks = P * 12, ts = P * (size_t)n_light * 48;
                dslot.probes = dbg->dump_probes;
                dslot.key = dbg->dump_key + (size_t)slot * ks;
                dslot.beta = dbg->dump_beta + (size_t)slot * ks;
                dslot.theta = dbg->dump_theta + (size_t)slot * ts;
                dslot.count = dbg->dump_count + (size_t)slot * ts;
                memset(dslot.key, 0, ks * sizeof(uint32_t));
                memset(dslot.beta, 0, ks * sizeof(double));
                memset(dslot.theta, 0, ts * sizeof(uint32_t));
                memset(dslot.count, 0, ts * sizeof(double));
                dd = &dslot;
            }
            if (load_pixel(gb, mats, n_mat, idx, &in, &lflags)) {
                shade_pixel(&in, &mats[in.mat], lights, n_light, prm, NULL, NULL, &o, dd);
            } else {
                memset(&o, 0, sizeof(o));
                o.flags = lflags;
                o.margin[0] = o.margin[1] = INFINITY;
            }
            for (int c = 0; c < 3; ++c) out_rgb[c * npx + idx] = o.rgb[c];
            if (dbg) {
                if (dbg->flags) dbg->flags[idx] = o.flags;
                if (dbg->n_probe) dbg->n_probe[idx] = o.n_probe;
                if (dbg->level) dbg->level[idx] = o.level;
                if (dbg->cell) dbg->cell[idx] = o.cell;
                if (dbg->key_sum) dbg->key_sum[idx] = o.key_sum;
                if (dbg->akey_sum) dbg->akey_sum[idx] = o.akey_sum;
                if (dbg->theta_sum) dbg->theta_sum[idx] = o.theta_sum;
                if (dbg->count_sum) dbg->count_sum[idx] = o.count_sum;
                if (dbg->n_open) dbg->n_open[idx] = o.n_open;
                if (dbg->n_gate) dbg->n_gate[idx] = o.n_gate;
                if (dbg->n_live) dbg->n_live[idx] = o.n_live;
                if (dbg->lit) dbg->lit[idx] = o.lit;
                if (dbg->margin) dbg->margin[idx] = o.margin[0];
                if (dbg->margin_kind) dbg->margin_kind[idx] = o.margin_kind[0];
                if (dbg->margin_pos) dbg->margin_pos[idx] = o.margin[1];
                if (dbg->margin_pos_kind) dbg->margin_pos_kind[idx] = o.margin_kind[1];
                if (dbg->b_light)
                    for (int li = 0; li < n_light; ++li) dbg->b_light[li * npx + idx] = o.b[li];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gradients of  sum_px sum_rgb g_rgb(px) L_rgb(px)  with respect to    */
/* each material's alpha and ln N and each light's raw direction, by   */
/* central differences of the relaxed forward (rounding 1).            */
/* frozen = 1: every light-dependent branch (light validity, p clamp,  */
/*   angular cell, gates, the max(1,x) clamp) is recorded at the base  */
/*   point and replayed at the shifted points: the derivative of the   */
/*   relaxed count with discrete branches held fixed.  The geometric   */
/*   decisions (probes, levels, cells, lattice) do not depend on these */
/*   parameters at all.                                                */
/* frozen = 0: plain central differences; a pixel whose branches flip  */
/*   between the base and a shifted point is left out and marked in    */
/*   flip[] (nullable).                                                */
/* grad_out: [3][height*stride] (double).  Outputs are overwritten.    */
/* The pixel sums are reduced row by row in a fixed order.             */
/* ------------------------------------------------------------------ */
static int same_tape(const og_tape *a, const og_tape *b)
{
    return a->len == b->len && memcmp(a->buf, b->buf, a->len * sizeof(int32_t)) == 0;
}

int og_grad(const og_gbuffer *gb, const og_material *mats, int n_mat, const og_light *lights,
            int n_light, const og_params *prm_in, const double *grad_out, double step,
            int frozen, double *g_alpha, double *g_lnN, double *g_dir, uint8_t *flip,
            int n_threads)
{
    if (!gb || !mats || n_mat <= 0 || n_light <= 0 || n_light > 64 || !grad_out || !(step > 0.0)) return -1;
    if (prm_in->count_law != 0) return -1;          /* the adjoint is the method's only */
    og_params prm = *prm_in;
    prm.rounding = 1;
    const int64_t npx = (int64_t)gb->height * gb->stride;
    const int np = 2 * n_mat + 3 * n_light;
    double *rows = (double *)calloc((size_t)np * (size_t)gb->height, sizeof(double));
    double *base_dirs = (double *)malloc(sizeof(double) * 3 * n_light);
    if (!rows || !base_dirs) { free(rows); free(base_dirs); return -2; }
    for (int li = 0; li < n_light; ++li)
        for (int c = 0; c < 3; ++c) base_dirs[3 * li + c] = lights[li].dir[c];
    set_threads(n_threads);
#pragma omp parallel
    {
        const int npp = 2 + 3 * n_light;           /* parameters seen by one pixel */
        double *dpx = (double *)malloc(sizeof(double) * npp);
        double *dirs_p = (double *)malloc(sizeof(double) * 3 * n_light);
        double *dirs_m = (double *)malloc(sizeof(double) * 3 * n_light);
        og_tape tb = {0}, tp = {0}, tm = {0};
#pragma omp for schedule(dynamic, 1)
        for (int y = 0; y < gb->height; ++y) {
            double *racc = rows + (size_t)y * np;
            for (int x = 0; x < gb->width; ++x) {
                int64_t idx = (int64_t)y * gb->stride + x;
                og_px_in in;
                uint32_t lflags = 0;
                if (flip) flip[idx] = 0;
                if (!load_pixel(gb, mats, n_mat, idx, &in, &lflags)) continue;
                const double go[3] = {grad_out[idx], grad_out[npx + idx], grad_out[2 * npx + idx]};
                og_px_out op, om;
                og_perturb pb = {0.0, 0.0, base_dirs};
                tb.len = 0; tb.pos = 0; tb.mode = 1;
                shade_pixel(&in, &mats[in.mat], lights, n_light, &prm, &pb, &tb, &op, NULL);
                if (!(op.flags & OGF_SHADED)) continue;
                int flipped = 0;
                for (int pi = 0; pi < npp; ++pi) {
                    memcpy(dirs_p, base_dirs, sizeof(double) * 3 * n_light);
                    memcpy(dirs_m, base_dirs, sizeof(double) * 3 * n_light);
                    og_perturb pp = {0.0, 0.0, dirs_p}, pm = {0.0, 0.0, dirs_m};
                    double hs;
                    if (pi == 0) { hs = step * in.alpha; pp.alpha_shift = hs; pm.alpha_shift = -hs; }
                    else if (pi == 1) { hs = step; pp.lnN_shift = hs; pm.lnN_shift = -hs; }
                    else { hs = step; dirs_p[pi - 2] += hs; dirs_m[pi - 2] -= hs; }
                    if (frozen) {
                        tb.mode = 2; tb.pos = 0;
                        shade_pixel(&in, &mats[in.mat], lights, n_light, &prm, &pp, &tb, &op, NULL);
                        tb.pos = 0;
                        shade_pixel(&in, &mats[in.mat], lights, n_light, &prm, &pm, &tb, &om, NULL);
                    } else {
                        tp.len = 0; tp.pos = 0; tp.mode = 1;
                        tm.len = 0; tm.pos = 0; tm.mode = 1;
                        shade_pixel(&in, &mats[in.mat], lights, n_light, &prm, &pp, &tp, &op, NULL);
                        shade_pixel(&in, &mats[in.mat], lights, n_light, &prm, &pm, &tm, &om, NULL);
                        if (!same_tape(&tp, &tb) || !same_tape(&tm, &tb)) flipped = 1;
                    }
                    double d = 0.0;
                    for (int c = 0; c < 3; ++c) d += go[c] * (op.rgb[c] - om.rgb[c]) / (2.0 * hs);
                    dpx[pi] = d;
                }
                if (flipped) { if (flip) flip[idx] = 1; continue; }
                racc[2 * in.mat] += dpx[0];
                racc[2 * in.mat + 1] += dpx[1];
                for (int i = 0; i < 3 * n_light; ++i) racc[2 * n_mat + i] += dpx[2 + i];
            }
        }
        free(dpx); free(dirs_p); free(dirs_m);
        free(tb.buf); free(tp.buf); free(tm.buf);
    }
    double *acc = (double *)calloc((size_t)np, sizeof(double));
    for (int y = 0; y < gb->height; ++y)
        for (int i = 0; i < np; ++i) acc[i] += rows[(size_t)y * np + i];
    for (int m = 0; m < n_mat; ++m) { g_alpha[m] = acc[2 * m]; g_lnN[m] = acc[2 * m + 1]; }
    for (int i = 0; i < 3 * n_light; ++i) g_dir[i] = acc[2 * n_mat + i];
    free(acc); free(rows); free(base_dirs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Forward-mode derivatives of the relaxed forward (dual numbers): a    */
/* second route to the gradient og_grad takes by central differences.  */
/* Every quantity that depends on a parameter carries its derivatives   */
/* with respect to the pixel's alpha (slot 0), its ln N (slot 1) and    */
/* the three raw direction components of the light being evaluated      */
/* (slots 2-4), through the same steps as shade_pixel (Eqs. 1-4, 10,    */
/* 14, 16-18; Schlick Fresnel, Smith masking).  Every discrete decision */
/* (light validity, p clamp, angular cell, gates, the max(1, x) clamp)  */
/* is taken on the values: the result is the derivative with those      */
/* decisions held fixed, as the adjoint defines it.                     */
/* ------------------------------------------------------------------ */
#define OGD_N 5
typedef struct { double v, d[OGD_N]; } ogd;

static ogd dconst(double v) { ogd r; r.v = v; for (int i = 0; i < OGD_N; ++i) r.d[i] = 0.0; return r; }
static ogd dvar(double v, int slot) { ogd r = dconst(v); r.d[slot] = 1.0; return r; }
static ogd dadd(ogd a, ogd b) { ogd r; r.v = a.v + b.v; for (int i = 0; i < OGD_N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
static ogd dsub(ogd a, ogd b) { ogd r; r.v = a.v - b.v; for (int i = 0; i < OGD_N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
static ogd dmul(ogd a, ogd b)
{
    ogd r;
    r.v = a.v * b.v;
    for (int i = 0; i < OGD_N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
static ogd ddiv(ogd a, ogd b)
{
    ogd r;
    r.v = a.v / b.v;
    for (int i = 0; i < OGD_N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
static ogd dscale(ogd a, double s) { for (int i = 0; i < OGD_N; ++i) a.d[i] *= s; a.v *= s; return a; }
static ogd daddc(ogd a, double c) { a.v += c; return a; }
/* f(a) with f(a.v) = fv and f'(a.v) = dfv (chain rule) */
static ogd dchain(ogd a, double fv, double dfv)
{
    ogd r;
    r.v = fv;
    for (int i = 0; i < OGD_N; ++i) r.d[i] = dfv * a.d[i];
    return r;
}
static ogd dsqrt(ogd a) { double s = sqrt(a.v); return dchain(a, s, 0.5 / s); }
static ogd dexp(ogd a) { double e = exp(a.v); return dchain(a, e, e); }
static ogd derf(ogd a) { return dchain(a, erf(a.v), 2.0 / sqrt(OG_PI) * exp(-a.v * a.v)); }
static ogd ddot3c(const ogd a[3], const double b[3])
{
    return dadd(dadd(dscale(a[0], b[0]), dscale(a[1], b[1])), dscale(a[2], b[2]));
}
/* a / |a|; 0 when the length is not finite and positive */
static int dnormalize3(ogd a[3])
{
    ogd l2 = dadd(dadd(dmul(a[0], a[0]), dmul(a[1], a[1])), dmul(a[2], a[2]));
    if (!(l2.v > 0.0) || !isfinite(l2.v)) return 0;
    ogd l = dsqrt(l2);
    for (int c = 0; c < 3; ++c) a[c] = ddiv(a[c], l);
    return 1;
}

/* og_ndf and og_smith_lambda with dual arguments (same formulas) */
static ogd d_ndf(int ndf, ogd alpha, ogd cm)
{
    if (cm.v <= 0.0) return dconst(0.0);
    ogd a2 = dmul(alpha, alpha), c2 = dmul(cm, cm);
    if (ndf == 0) {
        ogd d = daddc(dmul(c2, daddc(a2, -1.0)), 1.0);
        return ddiv(a2, dscale(dmul(d, d), OG_PI));
    }
    ogd tan2 = ddiv(dsub(dconst(1.0), c2), c2);
    return ddiv(dexp(dscale(ddiv(tan2, a2), -1.0)), dscale(dmul(a2, dmul(c2, c2)), OG_PI));
}

static ogd d_smith_g1(int ndf, ogd alpha, ogd c)
{
    ogd lam = dconst(0.0);
    if (c.v < 1.0) {
        ogd c2 = dmul(c, c);
        ogd tan2 = ddiv(dsub(dconst(1.0), c2), c2);
        if (ndf == 0) {
            lam = dscale(daddc(dsqrt(daddc(dmul(dmul(alpha, alpha), tan2), 1.0)), -1.0), 0.5);
        } else {
            ogd a = ddiv(dconst(1.0), dmul(alpha, dsqrt(tan2)));
            lam = dadd(dscale(daddc(derf(a), -1.0), 0.5),
                       ddiv(dexp(dscale(dmul(a, a), -1.0)), dscale(a, 2.0 * sqrt(OG_PI))));
        }
    }
    return ddiv(dconst(1.0), daddc(lam, 1.0));
}

/* one pixel: adds sum_rgb go_rgb L_rgb to *loss and its derivatives to
 * ga (alpha), gn (ln N) and gd[3 li + c] (light li's raw direction) */
static void grad_pixel_dual(const og_px_in *in, const og_material *mat, const og_light *lights, int n_light,
                            const og_params *prm, const double go[3], double *loss, double *ga, double *gn,
                            double *gd)
{
    double mgd[2] = {INFINITY, INFINITY};
    int mkd[2] = {MK_NONE, MK_NONE};
    const int K = prm->k_max;
    double nrm[3] = {in->n[0], in->n[1], in->n[2]};
    double wi[3] = {in->wi[0], in->wi[1], in->wi[2]};
    if (!normalize3(nrm) || !normalize3(wi)) return;
    double tt[3], bb[3];
    if (!tangent_frame(nrm, in->has_t ? in->t : NULL, tt, bb, mgd, mkd)) return;
    double P, r, phi, sigma0;
    if (!og_footprint(in->dudx, in->dvdx, in->dudy, in->dvdy, &P, &r, &phi, &sigma0)) return;
    const double cos_i = dot3(nrm, wi);
    if (!(cos_i > 0.0)) return;
    int n_pr = (int)ceil(r / ldexp(1.0, K));
    if (n_pr < 1) n_pr = 1;
    if (n_pr > prm->n_probe_max) n_pr = prm->n_probe_max;
    double Pk = P / n_pr, rk = r / n_pr;
    if (rk > ldexp(1.0, K)) rk = ldexp(1.0, K);
    og_nodes nodes;
    og_grid_nodes(Pk, rk, phi, K, &nodes, mgd, mkd);

    /* the probes' texel keys and weights do not depend on the parameters */
    enum { PMAX = 64 };
    static _Thread_local uint32_t pre[PMAX][OG_MAX_NODES][3];
    static _Thread_local double beta[PMAX][OG_MAX_NODES][3];
    const uint32_t s0 = og_hash_step(0x243F6A88u, mat->seed);
    for (int kp = 0; kp < n_pr && kp < PMAX; ++kp) {
        double cx, cy;
        probe_centre(in->u, in->v, phi, sigma0, n_pr, kp, &cx, &cy);
        for (int g = 0; g < nodes.n; ++g) {
            int vi[3], vj[3];
            og_simplex(cx, cy, nodes.l[g], nodes.k[g], nodes.m[g], vi, vj, beta[kp][g], mgd, mkd);
            uint32_t base = og_hash_step(s0, node_word(nodes.l[g], nodes.k[g], nodes.m[g]));
            for (int e = 0; e < 3; ++e)
                pre[kp][g][e] = og_hash_step(og_hash_step(base, (uint32_t)vi[e]), (uint32_t)vj[e]);
        }
    }

    const ogd alpha = dvar(in->alpha, 0);
    const ogd lnN = dvar(in->log10N * log(10.0), 1);
    const ogd N = dexp(lnN);
    const double R = mat->R;
    const ogd Dn = ddiv(dconst(1.0), dscale(dmul(alpha, alpha), OG_PI));
    const ogd cosi = dconst(cos_i);
    const ogd G1i = d_smith_g1(mat->ndf, alpha, cosi);
    const double mr = mat->micro_roughness;

    for (int li = 0; li < n_light; ++li) {
        ogd wo[3];
        for (int c = 0; c < 3; ++c) wo[c] = dvar((double)lights[li].dir[c], 2 + c);
        if (!dnormalize3(wo)) continue;
        const ogd cos_o = ddot3c(wo, nrm);
        if (!(cos_o.v > 0.0)) continue;
        ogd h[3];
        for (int c = 0; c < 3; ++c) h[c] = daddc(wo[c], wi[c]);
        if (!dnormalize3(h)) continue;
        const ogd cos_h = ddot3c(h, nrm);
        /* Eq. 4 */
        const ogd praw = ddiv(dscale(d_ndf(mat->ndf, alpha, cos_h), R), Dn);
        const ogd p = praw.v > 1.0 ? dconst(1.0) : praw;
        /* Eq. 14: the cell from the values, the weights as duals */
        const ogd ax = daddc(dscale(ddot3c(h, tt), 1.0 / mr), -0.5);
        const ogd ay = daddc(dscale(ddot3c(h, bb), 1.0 / mr), -0.5);
        const int ai = (int)floor(ax.v), aj = (int)floor(ay.v);
        const ogd fx = daddc(ax, -(double)ai), fy = daddc(ay, -(double)aj);
        const ogd gx = dsub(dconst(1.0), fx), gy = dsub(dconst(1.0), fy);
        ogd vw[4] = {dmul(gx, gy), dmul(fx, gy), dmul(gx, fy), dmul(fx, fy)};
        uint32_t ak[4][2];
        for (int a = 0; a < 4; ++a)
            for (int s = 0; s < 2; ++s)
                ak[a][s] = og_hash_step(0x13198A2Eu, angular_word(ai + (a & 1), aj + (a >> 1), s));
        /* Schlick Fresnel and Smith masking (Eq. 2) */
        const ogd ch = ddot3c(h, wi);
        const ogd om = dsub(dconst(1.0), ch);
        const ogd om2 = dmul(om, om);
        const ogd F = daddc(dscale(dmul(dmul(om2, om2), om), 1.0 - mat->F0), mat->F0);
        const ogd G = dmul(G1i, d_smith_g1(mat->ndf, alpha, cos_o));
        /* Eqs. 10, 16-18 over the probes, nodes, texels and angular texels */
        ogd bsum = dconst(0.0);
        for (int kp = 0; kp < n_pr && kp < PMAX; ++kp)
            for (int g = 0; g < nodes.n; ++g) {
                const ogd ng = dscale(N, nodes.w[g] * ldexp(1.0, nodes.l[g]));
                double pg;
                if (!(ng.v > 0.0) || !(p.v > 0.0)) pg = 0.0;
                else if (p.v >= 1.0) pg = 1.0;
                else pg = -expm1(ng.v * log1p(-p.v));
                const ogd mm = ng.v - 1.0 > 0.0 ? daddc(ng, -1.0) : dconst(0.0);
                const ogd mu = dmul(mm, p);
                const ogd var = dmul(mu, dsub(dconst(1.0), p));
                const ogd sg = var.v > 0.0 ? dsqrt(var) : dconst(0.0);
                for (int e = 0; e < 3; ++e)
                    for (int a = 0; a < 4; ++a) {
                        const uint32_t h0 = gate_word(prm, pre[kp][g][e], ak[a][0]);
                        if (!(uniform_of(h0) < pg)) continue;
                        const uint32_t h1 = gate_word(prm, pre[kp][g][e], ak[a][1]);
                        const double z = og_ndtri(uniform_of(h1));
                        const ogd x = daddc(dadd(mu, dscale(sg, z)), 1.0);
                        const ogd c = x.v >= 1.0 ? x : dconst(1.0);
                        bsum = dadd(bsum, dscale(dmul(vw[a], c), beta[kp][g][e]));
                    }
            }
        /* Eqs. 1-4 */
        const ogd DP = ddiv(dmul(Dn, bsum), dscale(N, R * P));
        const ogd f = dscale(dmul(dmul(F, G), DP), 1.0 / (4.0 * cos_i));
        double w = 0.0;
        for (int c = 0; c < 3; ++c) w += go[c] * (double)lights[li].radiance[c];
        *loss += w * f.v;
        *ga += w * f.d[0];
        *gn += w * f.d[1];
        for (int c = 0; c < 3; ++c) gd[3 * li + c] += w * f.d[2 + c];
    }
}

/* Gradients of  sum_px sum_rgb g_rgb(px) L_rgb(px)  (relaxed counts) by  */
/* forward-mode derivatives; same outputs as og_grad (frozen), plus the   */
/* loss itself.  Pixel sums are reduced row by row in a fixed order.     */
int og_grad_dual(const og_gbuffer *gb, const og_material *mats, int n_mat, const og_light *lights,
                 int n_light, const og_params *prm_in, const double *grad_out, double *g_alpha,
                 double *g_lnN, double *g_dir, double *loss_out, int n_threads)
{
    if (!gb || !mats || n_mat <= 0 || n_light <= 0 || n_light > 64 || !grad_out) return -1;
    if (prm_in->count_law != 0 || prm_in->n_probe_max > 64) return -1;
    og_params prm = *prm_in;
    prm.rounding = 1;
    const int64_t npx = (int64_t)gb->height * gb->stride;
    const int np = 2 * n_mat + 3 * n_light + 1;           /* the last column: the loss */
    double *rows = (double *)calloc((size_t)np * (size_t)gb->height, sizeof(double));
    if (!rows) return -2;
    set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < gb->height; ++y) {
        double *racc = rows + (size_t)y * np;
        for (int x = 0; x < gb->width; ++x) {
            const int64_t idx = (int64_t)y * gb->stride + x;
            og_px_in in;
            uint32_t lflags = 0;
            if (!load_pixel(gb, mats, n_mat, idx, &in, &lflags)) continue;
            const double go[3] = {grad_out[idx], grad_out[npx + idx], grad_out[2 * npx + idx]};
            grad_pixel_dual(&in, &mats[in.mat], lights, n_light, &prm, go, &racc[np - 1], &racc[2 * in.mat],
                            &racc[2 * in.mat + 1], &racc[2 * n_mat]);
        }
    }
    double *acc = (double *)calloc((size_t)np, sizeof(double));
    if (!acc) { free(rows); return -2; }
    for (int y = 0; y < gb->height; ++y)
        for (int i = 0; i < np; ++i) acc[i] += rows[(size_t)y * np + i];
    for (int m = 0; m < n_mat; ++m) { g_alpha[m] = acc[2 * m]; g_lnN[m] = acc[2 * m + 1]; }
    for (int i = 0; i < 3 * n_light; ++i) g_dir[i] = acc[2 * n_mat + i];
    if (loss_out) *loss_out = acc[np - 1];
    free(acc); free(rows);
    return 0;
}
