// glint_order.hip -- the tile-order pre-pass of glint_shade (and of the
// adjoint without lit masks): heaviest tiles first.  A translation unit of
// its own so that it is compiled with the default instruction scheduler (the
// shading kernels use one that trades registers for parallelism, which would
// make the single-workgroup scan spill).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "glint_device.hpp"
#include "glint_host.hpp"

namespace glint {

// ---------------------------------------------------------------------------
// Tile order for glint_shade: a stable counting sort of the tiles by cost
// class, heaviest class first, so that the long tiles (footprints split into
// many probes) start early instead of trailing at the end of the grid.  The
// order only schedules work; every tile's arithmetic is unchanged.
//   count:   tile cost S = sum of the pixels' probe counts (an FP32 estimate
//            of the forward's n_pr), class of ceil(S / 64) item batches (with
//            an even number of tile columns, the heavier class of the two
//            tiles that share the same 128-byte lines for both);
//            per block of kOrderTiles tiles, the count of each class
//   scan:    one workgroup turns the counts into output offsets
//   scatter: one workgroup per block ranks its tiles within each class; the
//            two tiles of such a pair get workgroups b and b + 8 (one XCD)
// ---------------------------------------------------------------------------
constexpr int kOrderClasses = 8;
constexpr int kOrderTiles = 64;       // tiles per count block
constexpr int kOrderWaves = 16;       // waves per count workgroup (4 tiles each)
constexpr int kScatterWaves = kOrderTiles / kWave;
constexpr int kScanThreads = 1024;

__device__ __forceinline__ int cost_class(int S)
{
    const int b = (S + kWave - 1) / kWave;
    return b < 4 ? b : (b < 6 ? 4 : (b < 9 ? 5 : (b < 14 ? 6 : 7)));
}

// probe count n_pr of a pixel as the forward computes it, in FP32 (an
// estimate: only the order of the tiles depends on it), from its derivatives
__device__ __forceinline__ int probe_estimate(float dux, float dvx, float duy, float dvy, float inv_rmax,
                                              int n_probe_max)
{
    const float a = dux * dux + duy * duy, b = dux * dvx + duy * dvy, c = dvx * dvx + dvy * dvy;
    const float P = fabsf(dux * dvy - duy * dvx);
    const float hd = 0.5f * (a - c);
    const float r = (0.5f * (a + c) + __builtin_amdgcn_sqrtf(hd * hd + b * b)) / P;
    const float n = ceilf(r * inv_rmax);
    return n >= 1.0f ? (n < (float)n_probe_max ? (int)n : n_probe_max) : 1;
}

__global__ __launch_bounds__(kWave * kOrderWaves) void glint_order_count(ViewDesc vw, int lw, int tiles_x, int32_t n_tiles,
                                                                         int n_mat, float inv_rmax,
                                                                         int n_probe_max, bool paired, uint8_t *cls,
                                                                         uint32_t *cnt)
{
    constexpr int kPerWave = kOrderTiles / kOrderWaves;
    __shared__ uint32_t s_cnt[kOrderWaves][kOrderClasses];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t t0 = (int64_t)blockIdx.x * kOrderTiles + w * kPerWave;
    // two rounds of loads for all the wave's tiles, each issued without
    // waiting: material ids, then derivatives.  Lanes outside the view or not
    // shaded read element 0 (the view is not empty) and drop the value.
    int64_t pix[kPerWave];
    bool in[kPerWave];
    int mat[kPerWave];
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        const int64_t t = t0 + i;
        const int x = ((int)(t % tiles_x) << lw) + (lane & ((1 << lw) - 1));
        const int y = ((int)(t / tiles_x) << (6 - lw)) + (lane >> lw);
        in[i] = t < n_tiles && x < vw.width && y < vw.height;
        pix[i] = in[i] ? (int64_t)y * vw.stride + x : 0;
    }
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        const int m = vw.mat ? vw.mat[pix[i]] : 0;
        mat[i] = in[i] ? m : -1;
    }
    float d[kPerWave][4];
    bool ok[kPerWave];
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        ok[i] = mat[i] >= 0 && mat[i] < n_mat;
        const int64_t q = ok[i] ? pix[i] : 0;
        d[i][0] = vw.dudx[q];
        d[i][1] = vw.dvdx[q];
        d[i][2] = vw.dudy[q];
        d[i][3] = vw.dvdy[q];
    }
    int S[kPerWave];
#pragma unroll
    for (int i = 0; i < kPerWave; ++i)
        S[i] = ok[i] ? probe_estimate(d[i][0], d[i][1], d[i][2], d[i][3], inv_rmax, n_probe_max) : 0;
    int c[kPerWave];
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        int v = S[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        c[i] = cost_class(v);
    }
    // paired: the two tiles of a pair (columns 2m and 2m + 1 of a row, the
    // two halves of the same 128-byte lines) take the heavier class, so that
    // they stay adjacent in the order (t0 is a multiple of 4, so pairs lie
    // inside the wave's tiles)
    if (paired) {
#pragma unroll
        for (int i = 0; i < kPerWave; i += 2) {
            const int m = c[i] > c[i + 1] ? c[i] : c[i + 1];
            c[i] = c[i + 1] = m;
        }
    }
    uint32_t mine = 0;                    // lane c < 8: this wave's count of class c
#pragma unroll
    for (int i = 0; i < kPerWave; ++i) {
        if (t0 + i < n_tiles) {
            if (lane == 0) cls[t0 + i] = (uint8_t)c[i];
            if (lane == c[i]) ++mine;
        }
    }
    if (lane < kOrderClasses) s_cnt[w][lane] = mine;
    __syncthreads();
    if (threadIdx.x < kOrderClasses) {
        uint32_t n = 0;
        for (int j = 0; j < kOrderWaves; ++j) n += s_cnt[j][threadIdx.x];
        cnt[(int64_t)blockIdx.x * kOrderClasses + threadIdx.x] = n;
    }
}

// counts cnt[block][class] -> offs[block][class]: class c's tiles of block b
// start at (tiles of heavier classes) + (class-c tiles of blocks before b).
// Each thread sums a contiguous run of blocks; the runs are scanned per
// class by DPP lane moves within each wave, then across the waves through
// one LDS exchange.
__global__ __launch_bounds__(kScanThreads) void glint_order_scan(const uint32_t *__restrict__ cnt,
                                                                 uint32_t *__restrict__ offs, int64_t n_blk)
{
    constexpr int kScanWaves = kScanThreads / kWave;
    __shared__ uint32_t s_wt[kOrderClasses][kScanWaves];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t per = (n_blk + kScanThreads - 1) / kScanThreads;
    const int64_t b0 = (int64_t)threadIdx.x * per < n_blk ? (int64_t)threadIdx.x * per : n_blk;
    const int64_t b1 = b0 + per < n_blk ? b0 + per : n_blk;
    uint32_t loc[kOrderClasses];
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c) loc[c] = 0;
    for (int64_t b = b0; b < b1; ++b)
#pragma unroll
        for (int c = 0; c < kOrderClasses; ++c) loc[c] += cnt[b * kOrderClasses + c];
    // exclusive prefix of this thread's run within its wave, per class
    uint32_t excl[kOrderClasses];
#pragma unroll
    for (int c = 0; c < kOrderClasses; ++c) {
        const uint32_t incl = (uint32_t)wave_inclusive_sum((int)loc[c]);
        if (lane == kWave - 1) s_wt[c][w] = incl;
        excl[c] = incl - loc[c];
    }
    __syncthreads();
    uint32_t base = 0, run[kOrderClasses];
#pragma unroll
    for (int c = kOrderClasses - 1; c >= 0; --c) {
        uint32_t tot = 0, pre = 0;
#pragma unroll
        for (int j = 0; j < kScanWaves; ++j) {
            const uint32_t x = s_wt[c][j];
            tot += x;
            pre += j < w ? x : 0u;
        }
        run[c] = base + pre + excl[c];
        base += tot;
    }
    for (int64_t b = b0; b < b1; ++b) {
        uint32_t n[kOrderClasses];
#pragma unroll
        for (int c = 0; c < kOrderClasses; ++c) n[c] = cnt[b * kOrderClasses + c];
#pragma unroll
        for (int c = 0; c < kOrderClasses; ++c) {
            offs[b * kOrderClasses + c] = run[c];
            run[c] += n[c];
        }
    }
}

__global__ __launch_bounds__(kOrderTiles) void glint_order_scatter(const uint8_t *__restrict__ cls,
                                                                   const uint32_t *__restrict__ offs,
                                                                   int32_t n_tiles, bool paired,
                                                                   int32_t *__restrict__ order)
{
    __shared__ uint32_t s_wc[kScatterWaves][kOrderClasses];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t t = (int64_t)blockIdx.x * kOrderTiles + threadIdx.x;
    const int c = t < n_tiles ? (int)cls[t] : -1;
    const uint64_t below = (1ull << lane) - 1ull;
    uint32_t rank = 0;
#pragma unroll
    for (int cc = 0; cc < kOrderClasses; ++cc) {
        const uint64_t m = __ballot(c == cc);
        if (c == cc) rank = (uint32_t)__popcll(m & below);
        if (lane == cc) s_wc[w][cc] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (c >= 0) {
        uint32_t pos = offs[(int64_t)blockIdx.x * kOrderClasses + c] + rank;
        for (int j = 0; j < w; ++j) pos += s_wc[j][c];
        // paired: position 16q + 2j + i (pair j of group q, member i) goes to
        // workgroup 16q + j + 8i, so that both tiles of a pair run on the same
        // XCD (workgroups go to the 8 XCDs in turn) at about the same time and
        // the second finds the shared lines in that XCD's L2; the last, partial
        // group of 16 keeps its positions
        if (paired && pos < ((uint32_t)n_tiles & ~15u)) pos = (pos & ~15u) + ((pos & 15u) >> 1) + ((pos & 1u) << 3);
        order[pos] = (int32_t)t;
    }
}

struct OrderLayout {
    int64_t n_tiles, n_blk;
    size_t cls_off, cnt_off, offs_off, bytes;
};

static OrderLayout order_layout(int32_t width, int32_t height)
{
    OrderLayout L;
    L.n_tiles = tiles_of(width, height);
    L.n_blk = (L.n_tiles + kOrderTiles - 1) / kOrderTiles;
    const size_t a = 256, cb = (size_t)L.n_blk * kOrderClasses * 4;
    L.cls_off = ((size_t)L.n_tiles * 4 + a - 1) / a * a;
    L.cnt_off = L.cls_off + ((size_t)L.n_blk * kOrderTiles + a - 1) / a * a;
    L.offs_off = L.cnt_off + (cb + a - 1) / a * a;
    L.bytes = L.offs_off + cb;
    return L;
}

size_t tile_order_bytes(int32_t width, int32_t height)
{
    if (width <= 0 || height <= 0) return 0;
    return order_layout(width, height).bytes;
}

int enqueue_tile_order(const ViewDesc &vw, const Shared &sh, void *ws, size_t ws_bytes, const int32_t **order,
                       hipStream_t st)
{
    const OrderLayout L = order_layout(vw.width, vw.height);
    if (ws_bytes < L.bytes || L.n_tiles > 0x7fffffffLL) return GLINT_ESHAPE;
    if ((uintptr_t)ws & 3u) return GLINT_EINVAL;
    const int tiles_x = (int)tiles_x_of(vw.width);
    char *w = (char *)ws;
    int32_t *ord = (int32_t *)w;
    uint8_t *cls = (uint8_t *)(w + L.cls_off);
    uint32_t *cnt = (uint32_t *)(w + L.cnt_off);
    uint32_t *offs = (uint32_t *)(w + L.offs_off);
    const float inv_rmax = 1.0f / (float)(1 << sh.k_max);
    const bool paired = (tiles_x & 1) == 0;   // every row splits into whole pairs
    hipLaunchKernelGGL(glint_order_count, dim3((unsigned)L.n_blk), dim3(kWave * kOrderWaves), 0, st, vw, kTileLw, tiles_x,
                       (int32_t)L.n_tiles, sh.n_mat, inv_rmax, sh.n_probe_max, paired, cls, cnt);
    hipLaunchKernelGGL(glint_order_scan, dim3(1), dim3(kScanThreads), 0, st, cnt, offs, L.n_blk);
    hipLaunchKernelGGL(glint_order_scatter, dim3((unsigned)L.n_blk), dim3(kOrderTiles), 0, st, cls, offs,
                       (int32_t)L.n_tiles, paired, ord);
    *order = ord;
    return GLINT_OK;
}

}  // namespace glint
