/*
 * glint.h -- C ABI of the MI355X (gfx950) per-pixel glint shading library.
 *
 * Method: Deliot & Belcour, "Real-Time Rendering of Glinty Appearances using
 * Distributed Binomial Laws on Anisotropic Grids" (HPG 2023).  For every pixel
 * of a G-buffer the library takes the UV footprint from the screen-space
 * derivatives (Sec. 5.1), picks the enclosing grids of the anisotropic
 * (area, ratio, orientation) grid family (Sec. 5.2, Eq. 13, Fig. 4, Sec. 6.1),
 * enumerates the simplex texels under the footprint (Sec. 6.2), hashes one
 * pair of uniforms per texel and angular texel, counts reflecting flakes with
 * the distributed gated binomial law (Eqs. 10, 14, 16-18) using
 * p = R D(h)/D(n) (Eq. 4), and returns the glint BRDF's radiance (Eqs. 1-3).
 *
 * Conventions shared by every entry point
 *  - Pointers inside glint_gbuffer, output arrays, gradients, workspaces and
 *    debug planes are DEVICE pointers on the current HIP device, owned by the
 *    caller.  glint_material / glint_light / glint_params / glint_tune
 *    arrays are HOST pointers; their contents are copied at the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously; no entry point synchronises.  Device
 *    faults surface at the caller's next synchronisation.
 *  - Return value: GLINT_OK (0) or a negative GLINT_E* status.  No exception
 *    crosses the ABI.  On GLINT_EHIP, glint_last_hip_error() gives the
 *    hipError_t of the failing call (per thread).
 *  - Planes are row-major [height][stride] with stride >= width (elements).
 *    out_rgb is SoA: three planes [3][height*stride] (R, G, B).
 *  - The library keeps no mutable global state except the static workspace
 *    of glint_shade_noalloc (one per GPU); it allocates device memory only
 *    inside glint_plan objects.
 */
#ifndef GLINT_H
#define GLINT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GLINT_OK = 0,
    GLINT_EINVAL = -1,        /* a parameter is out of its documented range        */
    GLINT_ENULL = -2,         /* a required pointer is NULL                        */
    GLINT_ESHAPE = -3,        /* width/height/stride/count inconsistent             */
    GLINT_EHIP = -4,          /* a HIP runtime call failed (glint_last_hip_error)  */
    GLINT_EUNSUPPORTED = -5,  /* valid request the library does not implement      */
    GLINT_ENOMEM = -6,        /* device allocation inside a plan failed            */
    GLINT_ELIMIT = -7         /* view larger than glint_shade_noalloc's static workspace */
};

#define GLINT_MAX_MATERIALS 32
#define GLINT_MAX_LIGHTS 16
#define GLINT_MAX_K 4              /* largest ratio level: r_max = 2^4 = 16 (Fig. 4)   */
#define GLINT_MAX_PROBES 64
#define GLINT_RNG_TABLE_MIN_LOG2 8   /* random-number table: 2^8 .. 2^32 words        */
#define GLINT_RNG_TABLE_MAX_LOG2 32
#define GLINT_RNG_LDS_MAX_LOG2 13    /* LDS placement: at most 2^13 words (32 KiB)     */
#define GLINT_RNG_CACHED 0           /* table read from device memory through L1/L2    */
#define GLINT_RNG_LDS 1              /* each tile's wave copies the table into LDS     */
#define GLINT_NOALLOC_WORKSPACE_BYTES 2097152  /* static workspace of glint_shade_noalloc, per GPU */
#define GLINT_TILE_W 16              /* glint_shade's tile: GLINT_TILE_W x GLINT_TILE_H pixels, */
#define GLINT_TILE_H 4               /* one 64-lane wave each                                 */

/* G-buffer of one view (Sec. 5.1 reads footprints from screen derivatives).
 * u, v: texture coordinates; dudx..dvdy: their screen-space derivatives
 * (the columns of J are d(uv)/dx and d(uv)/dy); n: shading normal; w: view
 * direction toward the eye (both normalised inside).  material_id < 0 skips
 * the pixel (output 0); material_id >= n_mat marks it invalid (output 0);
 * NULL material_id means material 0 everywhere.  alpha_px and
 * log10_density_px, when non-NULL, override the material's roughness and
 * flake density per pixel.  tx, ty, tz (all three or none; NULL: the
 * orthonormal basis of n of Duff et al. 2017) give a tangent per pixel whose
 * component orthogonal to n, normalised, is the first axis t of the angular
 * grid, with b = n x t (Sec. 5.2, Eq. 14); it need not be unit length.
 * Non-finite inputs, det J = 0, a view below the surface or a supplied
 * tangent within about 1e-3 rad of n (sin^2 of the angle below 1e-6) or of
 * zero length give output 0 (flag bit 3). */
typedef struct {
    int32_t width, height;
    int64_t stride;
    const float *u, *v, *dudx, *dvdx, *dudy, *dvdy;
    const float *nx, *ny, *nz, *wx, *wy, *wz;
    const int32_t *material_id;
    const float *alpha_px;
    const float *log10_density_px;
    const float *tx, *ty, *tz;
} glint_gbuffer;

/* Glint material (Sec. 3).  ndf: 0 GGX, 1 Beckmann.  alpha > 0: roughness of
 * D.  R in (0,1]: ratio of Eq. 4.  log10_density: flakes per unit UV area
 * (log10).  micro_roughness in [1e-4, 1]: angular cell size over the
 * orthographic projection of h (Eq. 14).  F0 in [0,1]: Schlick Fresnel at
 * normal incidence.  seed: selects the random numbers of the material. */
typedef struct {
    int32_t ndf;
    float alpha, R, log10_density, micro_roughness, F0;
    uint32_t seed;
} glint_material;

/* Directional light: dir points toward the light (normalised inside; the
 * gradient is taken with respect to the raw vector); radiance is RGB. */
typedef struct {
    float dir[3];
    float radiance[3];
} glint_light;

/* k_max in [0, 4]: largest ratio level of the grid family (0 = isotropic
 * grids only).  n_probe_max in [1, 64]: footprints with ratio above 2^k_max
 * are split into ceil(r / 2^k_max) sub-footprints, at most n_probe_max.
 * rounding: 0 = counts floor(1 + mu + sigma z) (Eq. 18); 1 = relaxed counts
 * max(1, 1 + mu + sigma z) (the function the backward differentiates).
 * flags: 0, or (glint_shade only) GLINT_FLAG_ZK_COUNT; every other entry
 * point rejects a nonzero value with EINVAL. */
typedef struct {
    int32_t k_max, n_probe_max, rounding;
    uint32_t flags;
} glint_params;

/* glint_params.flags bit: count with the prior-art law the method replaces
 * (Zirr and Kaplanyan; Sec. 2, Eq. 7 and Sec. 6.3, Eq. 15), an A/B baseline
 * on the same grids, texels and uniforms.  Grid node g counts its whole
 * cell, n = N 2^l_g trials: when n p > 5 or n > 16 the count of a texel is
 * max(0, floor(n p + sqrt(n p (1 - p)) Phi^-1(theta_0))), otherwise the
 * number of k in 1..floor(n + 1/2) whose uniform of H(h0, k) is below p
 * (h0 the texel's slot-0 word, theta_0 its uniform); the per-node outputs
 * are summed with the node weights w_g (a mix of outputs, Eq. 7, instead of
 * the distribution of trials, Eq. 10).  Requires rounding = 0.  Debug
 * planes then count: n_open the texels on the Gaussian branch, n_live the
 * Bernoulli trials drawn, count_sum the sum of the counts. */
#define GLINT_FLAG_ZK_COUNT 1u

/* Optional per-pixel debug planes of glint_shade (each [height*stride] or
 * NULL).  They hold exact integer fingerprints of every discrete decision, so
 * that a reference implementation can be compared bit for bit:
 *  flags      bit0 shaded, bit1 ratio clamped at n_probe_max, bit2 p clamped
 *             to 1, bit3 invalid input, bit4 view below surface, bit5 skipped
 *             (material_id < 0), bit6 material_id >= n_mat
 *  n_probe    number of sub-footprints; level: area level l = floor(log2 P_k)
 *  cell       kappa | j<<3 | triangle<<9 | pivot<<11 | D<<13 | n_nodes<<15
 *  key_sum    sum (mod 2^32) of the texel key hashes of every probe
 *  akey_sum   sum (mod 2^32) of the angular key hashes (slot 0) of every light
 *  theta_sum  sum (mod 2^32) of every gate hash (all 48 per probe and light)
 *  count_sum  sum of all integer counts (rounding 0)
 *  n_open     number of open gates; n_gate: number of gated binomials;
 *             n_live: gated binomials whose gate probability reaches the
 *             smallest uniform 2^-24 (the others cannot open)
 *  b_light    [n_light][height*stride] distributed count sum b per light
 *  n_live_small  live gated binomials whose gate threshold is below 2^16
 *             (gate probability at most 2^-16): the hash head decides them
 *             (work counter, no parity field)
 *  n_lit      (probe, light) pairs with at least one open gate: only these
 *             need the light's Fresnel, shadowing and radiance terms (work
 *             counter, no parity field)
 *  n_live_lit live gated binomials of those (probe, light) pairs: the gates
 *             the adjoint re-evaluates (work counter, no parity field)
 *
 * Sampled per-texel dump (dump_slot NULL: none).  dump_slot [height*stride]
 * names, per pixel, the slot s in [0, dump_capacity) that receives every
 * texel-level decision of the pixel, or -1 (any value outside that range is
 * ignored; two pixels naming one slot race).  A slot holds the pixel's probes
 * k < dump_probes (1 <= dump_probes <= GLINT_MAX_PROBES), and for each its
 * grid nodes g < 4 (Sec. 4.3), the three vertices e of the node's lattice
 * triangle (Sec. 6.2) and, per light l, the four angular texels a of Eq. 14
 * (a & 1 steps the angular x index, a >> 1 the y index):
 *  dump_key   [cap][dump_probes][4][3]        texel key: the hash chain of
 *             the material seed, the node's level, ratio and orientation
 *             words and the vertex's lattice indices (Sec. 5.1 seeds)
 *  dump_beta  [cap][dump_probes][4][3]        barycentric weight of the vertex
 *  dump_theta [cap][dump_probes][n_light][4][3][4]  slot-0 word h whose
 *             uniform (2 (h >> 9) + 1) 2^-24 decides the gate (Eq. 18); with
 *             GLINT_FLAG_ZK_COUNT the word behind the texel's count
 *  dump_count [cap][dump_probes][n_light][4][3][4]  count c of the texel
 *             (Eq. 17; 0 when the gate stays closed; the baseline's count
 *             with GLINT_FLAG_ZK_COUNT)
 * Entries of probes k >= n_probe, nodes beyond the pixel's node count, lights
 * below the pixel's horizon and pixels that are not shaded are written as 0
 * (every entry of a named slot is written).  All four arrays are required
 * with dump_slot; device memory, 4-byte aligned, owned by the caller. */
typedef struct {
    uint32_t *flags;
    int32_t *n_probe, *level;
    uint32_t *cell, *key_sum, *akey_sum, *theta_sum, *count_sum, *n_open, *n_gate, *n_live;
    float *b_light;
    uint32_t *n_live_small, *n_lit, *n_live_lit;
    const int32_t *dump_slot;
    int32_t dump_capacity, dump_probes;
    uint32_t *dump_key;
    float *dump_beta;
    uint32_t *dump_theta;
    float *dump_count;
} glint_debug;

/* Launch configuration of the batched path (autotuner output).
 * tile_w x tile_h pixels per work unit (tile_w*tile_h == 64 * waves);
 * blocks_per_cu in [1, 64]: persistent workgroups per compute unit that pop
 * chunks of tiles from a counter; 0: one workgroup per tile (the grid covers
 * the whole tile table, each workgroup finds its view by binary search). */
typedef struct {
    int32_t tile_w, tile_h, blocks_per_cu, reserved;
} glint_tune;

typedef struct glint_plan glint_plan;

/* Workspace of glint_shade for a width x height view, in bytes (0 when the
 * view is empty): about 5.5 bytes per 64-pixel tile. */
size_t glint_shade_workspace_bytes(int32_t width, int32_t height);

/* Forward shading of one view: out_rgb[3][height*stride] <- radiance
 * L = sum_l E_l F G D_P / (4 <w,n>) with D_P = D(n) b / (R N P)
 * (Eqs. 1-4, 10, 14, 16-18).  n_mat in [1, 32], n_light in [0, 16].
 * With params->flags = GLINT_FLAG_ZK_COUNT b is the baseline's mixed count
 * instead (Eqs. 7 and 15; see that flag).
 * dbg may be NULL.
 * workspace: device memory of at least glint_shade_workspace_bytes(width,
 * height) bytes, 4-byte aligned, owned by the caller and used by this call
 * only (calls that overlap on the device need their own).  The view is
 * shaded in tiles of GLINT_TILE_W x GLINT_TILE_H = 16 x 4 pixels (one
 * 64-lane wave each; n_tiles = ceil(width/16) * ceil(height/4)).  With a workspace the tiles are shaded
 * heaviest first (a cost pre-pass over the derivatives orders them by their
 * number of probe items; the first 4*n_tiles bytes then hold that order as
 * int32 tile indices, row-major tile numbering); with workspace == NULL they
 * are shaded in row-major order.
 * The image is bit-identical either way.
 * Errors: ENULL (gbuf, planes, mats, out_rgb, lights when n_light > 0, a
 * dump array when dbg->dump_slot is set),
 * ESHAPE (width/height < 0, stride < width, workspace_bytes too small),
 * EINVAL (params or material values out of range, misaligned workspace,
 * dump_capacity < 1, dump_probes outside [1, GLINT_MAX_PROBES], misaligned
 * dump arrays),
 * EHIP (launch failure). */
int glint_shade(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                const glint_light *lights, int32_t n_light, const glint_params *params,
                float *out_rgb, const glint_debug *dbg, void *workspace, size_t workspace_bytes,
                void *stream);

/* glint_shade that also records, for the adjoint, which lights and which
 * probes opened at least one gate (Eq. 18) in each pixel: bit l of
 * lit_lights[y*stride + x] is set iff some gate of light l opened in some
 * probe of the pixel; bit k of lit_probes[y*stride + x] iff some gate opened
 * in probe k (bit 31: in probe 31 or a later one); both 0 for pixels that
 * are not shaded.  The radiance equals glint_shade's bit for bit.
 * lit_lights: device memory of height*stride uint16 values, 2-byte aligned;
 * lit_probes (nullable): height*stride uint32 values, 4-byte aligned; both
 * owned by the caller, overwritten.  Errors as glint_shade, plus ENULL
 * (lit_lights), EINVAL (misaligned lit_lights or lit_probes). */
int glint_shade_lit(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                    const glint_light *lights, int32_t n_light, const glint_params *params,
                    float *out_rgb, uint16_t *lit_lights, uint32_t *lit_probes, void *workspace,
                    size_t workspace_bytes, void *stream);

/* glint_shade for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same heaviest-first shading as glint_shade with a workspace, the
 * same image bit for bit, but the tile-order workspace is a static device
 * array of the library (GLINT_NOALLOC_WORKSPACE_BYTES = 2 MiB on every GPU
 * the library runs on, held until the process ends).  The call allocates
 * nothing and takes no debug planes; the caller still owns gbuf and out_rgb.
 * Every call on one GPU uses that GPU's single array: calls that overlap on
 * one device (two streams, two host threads) race and must be serialised by
 * the caller; consecutive calls on one stream are safe (each rewrites what it
 * reads).  The first call on a device looks up the array's address on that
 * device (hipGetSymbolAddress) and caches it.
 * Errors as glint_shade, plus ELIMIT when glint_shade_workspace_bytes(width,
 * height) exceeds GLINT_NOALLOC_WORKSPACE_BYTES (about 22 million pixels,
 * e.g. 5120 x 4096 fits, 8192 x 4096 does not), EUNSUPPORTED when the current
 * device index is 64 or above. */
int glint_shade_noalloc(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                        const glint_light *lights, int32_t n_light, const glint_params *params,
                        float *out_rgb, void *stream);

/* Random-number table for glint_shade_rng_table (Sec. 6.3: the two uniforms
 * of a gated binomial may be read from a small texture of random numbers
 * precomputed once): table[i] = H(seed, i) for i < 2^log2_words, with
 * H(h, w) = fmix32((h ^ w) + 0x9E3779B9) and fmix32 the MurmurHash3
 * finaliser, enqueued on stream.  table: device memory of 4 * 2^log2_words
 * bytes, 16-byte aligned, owned by the caller.  log2_words in [8, 32].
 * Errors: ENULL (table), EINVAL (log2_words out of range, misaligned
 * table), EHIP (launch failure). */
int glint_rng_table_fill(uint32_t *table, int32_t log2_words, uint32_t seed, void *stream);

/* glint_shade with the gate and count uniforms read from a random-number
 * table instead of hashed (Sec. 6.3, the precomputed texture): the word of
 * (texel key t, angular key a) is table[(t ^ a) & (2^log2_words - 1)]
 * instead of H(t, a); everything else is glint_shade's.  With a table
 * filled by glint_rng_table_fill(table, 32, 0) the result equals
 * glint_shade's bit for bit (table[i] = H(0, i) and H(0, t ^ a) = H(t, a)).
 * table: device memory of 2^log2_words words (any contents), 16-byte
 * aligned, owned by the caller, read only.  placement: GLINT_RNG_CACHED
 * reads the table from device memory through the caches (log2_words in
 * [8, 32]); GLINT_RNG_LDS copies it into each tile's LDS first (log2_words
 * in [8, 13], 4 * 2^log2_words bytes of LDS per 64-pixel tile, which lowers
 * occupancy).  Both placements give the same image; dbg (as glint_shade's)
 * is produced by the instrumented kernel, which reads the table through the
 * caches.  Errors as glint_shade, plus ENULL (table), EINVAL (placement,
 * log2_words out of range for the placement, misaligned table). */
int glint_shade_rng_table(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                          const glint_light *lights, int32_t n_light, const glint_params *params,
                          const uint32_t *table, int32_t log2_words, int32_t placement,
                          float *out_rgb, const glint_debug *dbg, void *workspace,
                          size_t workspace_bytes, void *stream);

/* Workspace for glint_shade_backward, in bytes. */
size_t glint_backward_workspace_bytes(int32_t width, int32_t height, int32_t n_mat, int32_t n_light);

/* Adjoint of the relaxed forward (rounding forced to 1): given
 * grad_out_rgb = dLoss/dL ([3][height*stride]), writes (overwriting)
 *   grad_alpha[n_mat]       dLoss/d alpha of each material
 *   grad_ln_density[n_mat]  dLoss/d ln N of each material
 *   grad_light_dir[3*n_light] dLoss/d dir (raw, unnormalised) of each light
 * Every discrete branch (level, cell, triangle, tetrahedron, lattice,
 * angular cell, gate, the max(1,.) clamp) is held at its value at the
 * current parameters.  Gradients are accumulated in FP32 per pixel and
 * reduced in a fixed order (deterministic).  Per-pixel overrides
 * (alpha_px, log10_density_px) are not supported (EUNSUPPORTED).
 * workspace: device memory of at least glint_backward_workspace_bytes()
 * bytes (about 4 bytes per pixel plus one partial row per 16x4 tile, or
 * per unit workgroup for small images),
 * 8-byte aligned, owned by the caller and used by this call only (tile
 * order, partial rows, FP64 reduction stage, lit-pixel list).  Without a
 * mask, tiles run heaviest first; the sums are reduced in a fixed order over
 * tiles, so the result does not depend on the schedule.
 * lit_lights, lit_probes (nullable): the masks glint_shade_lit wrote for
 * the same inputs with rounding 1 (relaxed; the gates do not depend on the
 * rounding).  lit_probes is used only with lit_lights.
 * Every gradient term of a light vanishes when none of its gates opened, so
 * only the pixels with a non-zero mask are shaded, and only their lights
 * with a set bit: a fraction of the work, the same terms summed in another
 * grouping (equal within FP32 rounding to the call without the mask;
 * deterministic).  With lit_lights alone the lit pixels are gathered in
 * raster order into waves of 64 (each chunk has its own partial row).  With
 * both masks (and n_light > 0) the work is cut into units of 64
 * (pixel, lit probe, lit light) items, one light per lane (bit 31 of the
 * probe mask stands for probes 31 to n_pr - 1), and 16384 workgroups take
 * equal contiguous ranges of units, each with its own partial row.  NULL
 * evaluates every gate of every pixel.  Errors as glint_shade, plus ENULL
 * (workspace, gradient outputs), EINVAL (misaligned workspace, lit_lights
 * or lit_probes). */
int glint_shade_backward(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                         const glint_light *lights, int32_t n_light, const glint_params *params,
                         const float *grad_out_rgb, const uint16_t *lit_lights,
                         const uint32_t *lit_probes, float *grad_alpha, float *grad_ln_density,
                         float *grad_light_dir, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Batched shading of many views of uneven size in one launch.
 * glint_plan_create copies the view descriptors (device pointers inside
 * gbufs/out_rgb stay owned by the caller and must outlive the plan), the
 * materials, lights and params, builds the tile table on the device, and
 * (tune may be NULL: 16 x 4 tiles, one workgroup per tile) fixes the launch
 * shape.
 * glint_shade_batched enqueues [counter reset kernel, persistent kernel]
 * (or, with blocks_per_cu = 0, one kernel with a workgroup per tile) on
 * `stream`; with use_graph != 0 it captures them once into a hipGraph and
 * replays the graph afterwards.  Each view's output is bit-identical to
 * glint_shade on that view.  The plan must not be used by two streams at
 * once (its tile counter is shared). */
int glint_plan_create(const glint_gbuffer *gbufs, float *const *out_rgb, int32_t n_views,
                      const glint_material *mats, int32_t n_mat, const glint_light *lights,
                      int32_t n_light, const glint_params *params, const glint_tune *tune,
                      glint_plan **plan);
int glint_shade_batched(glint_plan *plan, int32_t use_graph, void *stream);
int glint_plan_destroy(glint_plan *plan);
/* number of tiles and of workgroups of a plan (for reports) */
int glint_plan_info(const glint_plan *plan, int64_t *n_tiles, int32_t *n_blocks);

/* The per-texel random numbers, for bit-exact checks: keys is a device array
 * [n][9] of int32 (seed, l, k, m, i, j, ai, aj, slot); out[n] receives the
 * 32-bit hash whose top 23 bits give the uniform (2 (h >> 9) + 1) 2^-24. */
int glint_texel_hash(const int32_t *keys, int64_t n, uint32_t *out, void *stream);

/* One hash chaining step H(h, w) on device arrays (bit-exact checks). */
int glint_hash_step(const uint32_t *h, const uint32_t *w, int64_t n, uint32_t *out, void *stream);

/* Standard normal inverse CDF of the FP32 path, evaluated at the uniform
 * (2 (bits >> 9) + 1) 2^-24 that each 32-bit hash word stands for. */
int glint_ndtri(const uint32_t *bits, int64_t n, float *out, void *stream);

const char *glint_status_string(int status);
int glint_last_hip_error(void);
/* ABI version: major*10000 + minor*100 + patch */
int glint_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GLINT_H */
