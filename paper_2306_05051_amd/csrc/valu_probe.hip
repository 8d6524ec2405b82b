// valu_probe.hip -- VALU issue rates of gfx950 per instruction class.
//
// Every kernel runs 8 independent loop-carried chains per lane, 64 copies of
// one instruction per loop trip (the loop body holds nothing else, which the
// compiled ISA shows), with 16 waves per SIMD; one extra run of the plain
// FP32 multiply uses one wave per SIMD.  Rates are printed as wavefront
// instructions per clock per SIMD at the 2.4 GHz peak engine clock, and as
// lane-operations per second.  The glint path's VALU roofline (its issue-slot
// costs and peak) is derived from these figures.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 8;

template <int OP>
__global__ __launch_bounds__(256) void chain_kernel(unsigned *out, unsigned seed, int iters)
{
    unsigned u[kChains];
    float f[kChains];
    double d[kChains];
    const unsigned t = threadIdx.x + blockIdx.x * 977u + seed;
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
        u[c] = t * (2u * c + 1u);
        f[c] = 1.0f + 1e-3f * (float)(t & 1023u) + (float)c;
        d[c] = (double)f[c];
    }
    const float mf = 0.999f + 1e-9f * (float)seed;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int s = 0; s < 64 / kChains; ++s) {
#pragma unroll
            for (int c = 0; c < kChains; ++c) {
                const int n = (c + 1) % kChains;
                if constexpr (OP == 0) f[c] = f[c] * f[n];                          // v_mul_f32
                if constexpr (OP == 1) f[c] = fmaf(f[c], mf, f[n]);                 // v_fma_f32
                if constexpr (OP == 2) u[c] = u[c] + u[n];                          // v_add_u32
                if constexpr (OP == 3) u[c] = u[c] * u[n];                          // v_mul_lo_u32
                if constexpr (OP == 4) d[c] = fma(d[c], (double)mf, d[n]);          // v_fma_f64
                if constexpr (OP == 5) d[c] = d[c] * d[n];                          // v_mul_f64
                if constexpr (OP == 6) f[c] = __builtin_amdgcn_exp2f(f[c]);         // v_exp_f32
                if constexpr (OP == 7) f[c] = __builtin_amdgcn_sqrtf(f[c]);         // v_sqrt_f32
                if constexpr (OP == 8) d[c] = __builtin_amdgcn_rsq(d[c]);           // v_rsq_f64
                if constexpr (OP == 9) d[c] = __builtin_amdgcn_rcp(d[c]);           // v_rcp_f64
            }
        }
    }
    unsigned acc = 0u;
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc ^= u[c] ^ __float_as_uint(f[c]) ^ (unsigned)__double2loint(d[c]);
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int OP>
int run(const char *name, unsigned *buf, int blocks, int iters)
{
    hipEvent_t s, e;
    if (hipEventCreate(&s) != hipSuccess || hipEventCreate(&e) != hipSuccess) return 1;
    float best = 1e30f;
    for (int r = 0; r < 3; ++r) {
        (void)hipEventRecord(s, 0);
        hipLaunchKernelGGL(chain_kernel<OP>, dim3(blocks), dim3(256), 0, 0, buf, 1u, iters);
        (void)hipEventRecord(e, 0);
        if (hipEventSynchronize(e) != hipSuccess) return 1;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, s, e);
        if (ms < best) best = ms;
    }
    (void)hipEventDestroy(s);
    (void)hipEventDestroy(e);
    const double waves = blocks * 4.0, inst = waves * iters * 64.0;
    std::printf("%-14s waves/SIMD %5.1f  %8.3f ms  %6.3f wave-inst/clk/SIMD  %7.2f T lane-op/s\n", name,
                waves / 1024.0, best, inst / (best * 1e-3) / 1024.0 / 2.4e9, inst * 64.0 / (best * 1e-3) / 1e12);
    return 0;
}

}  // namespace

int main()
{
    const int full = 256 * 16, one = 256;      // workgroups of 4 waves: 16 and 1 waves per SIMD on 256 CUs
    unsigned *buf = nullptr;
    if (hipMalloc((void **)&buf, sizeof(unsigned) * (size_t)full * 256) != hipSuccess) return 1;
    int rc = 0;
    rc |= run<0>("v_mul_f32", buf, one, 16000);
    rc |= run<0>("v_mul_f32", buf, full, 1000);
    rc |= run<1>("v_fma_f32", buf, full, 1000);
    rc |= run<2>("v_add_u32", buf, full, 1000);
    rc |= run<3>("v_mul_lo_u32", buf, full, 1000);
    rc |= run<4>("v_fma_f64", buf, full, 1000);
    rc |= run<5>("v_mul_f64", buf, full, 1000);
    rc |= run<6>("v_exp_f32", buf, full, 500);
    rc |= run<7>("v_sqrt_f32", buf, full, 500);
    rc |= run<8>("v_rsq_f64", buf, full, 250);
    rc |= run<9>("v_rcp_f64", buf, full, 250);
    (void)hipFree(buf);
    return rc;
}
