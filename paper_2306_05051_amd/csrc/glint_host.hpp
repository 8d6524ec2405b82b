// glint_host.hpp -- host-side helpers shared by the library's translation
// units: argument validation, kernel-argument preparation, error state.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/glint.h"
#include "glint_device.hpp"

namespace glint {

int set_hip_error(hipError_t e);   // records e for glint_last_hip_error, returns GLINT_EHIP

// Tile shape of glint_shade and glint_shade_backward: kTileW x kTileH pixels
// per 64-lane wave.  16 x 4 tiles (half a 128-byte cache line per G-buffer
// plane and row) are 2.3% faster on the 4K frame than 32 x 2 (whole lines)
// and 8 x 8: the more compact the tile, the more its items share their
// lights' angular cells and their gates' liveness, and the G-buffer reads
// are not what bounds the kernel.
constexpr int kTileLw = 4;
constexpr int kTileW = 1 << kTileLw, kTileH = kWave / kTileW;
static_assert(kTileW == GLINT_TILE_W && kTileH == GLINT_TILE_H, "tile shape of the header");

inline int64_t tiles_x_of(int32_t width) { return (width + kTileW - 1) / kTileW; }
inline int64_t tiles_of(int32_t width, int32_t height)
{
    return tiles_x_of(width) * (int64_t)((height + kTileH - 1) / kTileH);
}

// Heaviest-first order of the kTileW x kTileH tiles of a view (row-major tile numbering),
// built on `st` in `ws` (tile_order_bytes(width, height) bytes, 4-byte
// aligned).  On success *order points at n_tiles int32 tile indices inside
// ws.  Defined in glint_order.hip.
size_t tile_order_bytes(int32_t width, int32_t height);
int enqueue_tile_order(const ViewDesc &vw, const Shared &sh, void *ws, size_t ws_bytes, const int32_t **order,
                       hipStream_t st);

inline bool finite_host(float x) { return std::isfinite(x); }

// Validates materials / lights / params and fills the kernel-argument block.
// allowed_flags: the params.flags bits the calling entry point accepts.
inline int prepare_shared(const glint_material *mats, int32_t n_mat, const glint_light *lights,
                          int32_t n_light, const glint_params *prm, Shared &sh, uint32_t allowed_flags = 0u)
{
    if (!mats || !prm || (n_light > 0 && !lights)) return GLINT_ENULL;
    if (n_mat < 1 || n_mat > kMaxMat || n_light < 0 || n_light > kMaxLight) return GLINT_EINVAL;
    if (prm->k_max < 0 || prm->k_max > GLINT_MAX_K || prm->n_probe_max < 1 ||
        prm->n_probe_max > GLINT_MAX_PROBES || (prm->rounding != 0 && prm->rounding != 1) ||
        (prm->flags & ~allowed_flags) != 0u)
        return GLINT_EINVAL;
    if ((prm->flags & GLINT_FLAG_ZK_COUNT) && prm->rounding != 0) return GLINT_EINVAL;   // integer counts
    std::memset(&sh, 0, sizeof(sh));
    for (int i = 0; i < n_mat; ++i) {
        const glint_material &m = mats[i];
        if ((m.ndf != 0 && m.ndf != 1) || !finite_host(m.alpha) || !(m.alpha > 0.0f) ||
            !finite_host(m.R) || !(m.R > 0.0f) || !(m.R <= 1.0f) || !(m.log10_density >= -20.0f) ||
            !(m.log10_density <= 20.0f) ||
            !(m.micro_roughness >= 1e-4f) || !(m.micro_roughness <= 1.0f) || !(m.F0 >= 0.0f) ||
            !(m.F0 <= 1.0f))
            return GLINT_EINVAL;
        DevMaterial &d = sh.mats[i];
        d.ndf = m.ndf;
        d.alpha = m.alpha;
        d.R = m.R;
        d.log10N = m.log10_density;
        d.F0 = m.F0;
        d.root = fmix32((kRootSalt ^ m.seed) + 0x9E3779B9u);
        d.inv_micro = 1.0 / (double)m.micro_roughness;
    }
    for (int i = 0; i < n_light; ++i) {
        const glint_light &l = lights[i];
        double w[3] = {l.dir[0], l.dir[1], l.dir[2]};
        double len = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        DevLight &d = sh.lights[i];
        d.ok = (len > 0.0 && std::isfinite(len)) ? 1 : 0;
        d.inv_len = d.ok ? (float)(1.0 / len) : 0.0f;
        for (int c = 0; c < 3; ++c) {
            d.wo[c] = d.ok ? w[c] / len : 0.0;
            if (!finite_host(l.radiance[c])) return GLINT_EINVAL;
            d.rad[c] = l.radiance[c];
        }
    }
    for (int m = 0; m < 32; ++m) {
        const double a = (double)m * 3.14159265358979323846 / 32.0;
        sh.cs[m][0] = std::cos(a);
        sh.cs[m][1] = std::sin(a);
    }
    sh.n_mat = n_mat;
    sh.n_light = n_light;
    sh.k_max = prm->k_max;
    sh.n_probe_max = prm->n_probe_max;
    sh.rounding = prm->rounding;
    return GLINT_OK;
}

inline int make_view(const glint_gbuffer *g, float *out, ViewDesc &v)
{
    if (!g) return GLINT_ENULL;
    if (g->width < 0 || g->height < 0 || g->stride < g->width) return GLINT_ESHAPE;
    if ((int64_t)g->width * g->height > 0) {
        if (!g->u || !g->v || !g->dudx || !g->dvdx || !g->dudy || !g->dvdy || !g->nx || !g->ny || !g->nz ||
            !g->wx || !g->wy || !g->wz || !out)
            return GLINT_ENULL;
    }
    v.width = g->width;
    v.height = g->height;
    v.stride = g->stride;
    v.u = g->u; v.v = g->v; v.dudx = g->dudx; v.dvdx = g->dvdx; v.dudy = g->dudy; v.dvdy = g->dvdy;
    v.nx = g->nx; v.ny = g->ny; v.nz = g->nz; v.wx = g->wx; v.wy = g->wy; v.wz = g->wz;
    v.mat = g->material_id;
    v.alpha_px = g->alpha_px;
    v.log10N_px = g->log10_density_px;
    v.out = out;
    // tangent planes: all three or none
    if ((g->tx || g->ty || g->tz) && !(g->tx && g->ty && g->tz)) return GLINT_ENULL;
    v.tx = g->tx;
    v.ty = g->ty;
    v.tz = g->tz;
    return GLINT_OK;
}

}  // namespace glint
