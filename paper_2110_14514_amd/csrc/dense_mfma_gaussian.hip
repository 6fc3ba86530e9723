// Matrix-core tile kernels instantiated for the gaussian loss.
#include "mfma_tile.hpp"

namespace gcp {

hipError_t dense_mfma_launch_gaussian(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                   float* gsp, float* lossp) {
  return by_rank<kGaussian>(c, p, G1p, G2p, G3p, gsp, lossp);
}

hipError_t dense_mfma_launch_gaussian_id(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p,
                                         float* G3p, float* gsp, float* lossp) {
  return by_rank<kGaussianId>(c, p, G1p, G2p, G3p, gsp, lossp);
}

void batch_launch_gaussian(const BatchRun& b, int v, int want, hipStream_t st) { launch_batch_loss<kGaussian>(b, v, want, st); }

}  // namespace gcp
