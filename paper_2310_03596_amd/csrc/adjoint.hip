// Hand-written adjoint of the fluid step (reverse of steps e and g).
#include "pair.hpp"

namespace sph {

namespace {

template <typename real>
__global__ __launch_bounds__(kBlock) void k_permute(uint32_t n, const uint32_t *__restrict__ perm, AV<real> in,
                                                    AV<real> out)
{
    uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    uint32_t d = perm[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (in.x[a]) out.x[a][d] = in.x[a][k];
        if (in.v[a]) out.v[a][d] = in.v[a][k];
    }
    if (in.m) out.m[d] = in.m[k];
    if (in.w) out.w[d] = in.w[k];
    if (in.E) out.E[d] = in.E[k];
}

}  // namespace

hipError_t launch_interact_adjoint(const Params &, const Grid &, int, const sph_particles &, const uint32_t *,
                                   const sph_rates &, const sph_adjoint &, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_integrate_adjoint(const Params &, int, int, const sph_particles &, const sph_rates &,
                                    const double *, const sph_adjoint &, const sph_rates &, double *,
                                    const Workspace &, hipStream_t)
{
    return hipErrorNotSupported;
}

hipError_t launch_permute_adjoint(int prec, uint32_t n, const uint32_t *perm, const sph_adjoint &in,
                                  const sph_adjoint &out, hipStream_t s)
{
    uint32_t blocks = div_up(n, kBlock);
    if (prec == SPH_FP64)
        k_permute<double><<<blocks, kBlock, 0, s>>>(n, perm, view<double>(in), view<double>(out));
    else
        k_permute<float><<<blocks, kBlock, 0, s>>>(n, perm, view<float>(in), view<float>(out));
    return hipGetLastError();
}

}  // namespace sph
