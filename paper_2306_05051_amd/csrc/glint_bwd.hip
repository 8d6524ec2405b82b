// glint_bwd.hip -- adjoint of the relaxed forward (placeholder until the
// adjoint kernel lands; reports EUNSUPPORTED).
#include <hip/hip_runtime.h>

#include "glint_host.hpp"

extern "C" {

size_t glint_backward_workspace_bytes(int32_t width, int32_t height, int32_t n_mat, int32_t n_light)
{
    (void)width; (void)height; (void)n_mat; (void)n_light;
    return 0;
}

int glint_shade_backward(const glint_gbuffer *gbuf, const glint_material *mats, int32_t n_mat,
                         const glint_light *lights, int32_t n_light, const glint_params *params,
                         const float *grad_out_rgb, float *grad_alpha, float *grad_ln_density,
                         float *grad_light_dir, void *workspace, size_t workspace_bytes, void *stream)
{
    (void)gbuf; (void)mats; (void)n_mat; (void)lights; (void)n_light; (void)params; (void)grad_out_rgb;
    (void)grad_alpha; (void)grad_ln_density; (void)grad_light_dir; (void)workspace; (void)workspace_bytes;
    (void)stream;
    return GLINT_EUNSUPPORTED;
}

}  // extern "C"
