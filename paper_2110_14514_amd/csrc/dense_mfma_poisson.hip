// Matrix-core tile kernels instantiated for the poisson loss.
#include "mfma_tile.hpp"

namespace gcp {

hipError_t dense_mfma_launch_poisson(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                  float* gsp, float* lossp) {
  return by_rank<kPoissonLog>(c, p, G1p, G2p, G3p, gsp, lossp);
}

void batch_launch_poisson(const BatchRun& b, int v, int want, hipStream_t st) { launch_batch_loss<kPoissonLog>(b, v, want, st); }

}  // namespace gcp
