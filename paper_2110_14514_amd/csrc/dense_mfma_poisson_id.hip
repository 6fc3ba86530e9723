// Matrix-core tile kernels instantiated for the poisson id loss (single streams;
// batches take the three log/logit/Gaussian losses).
#include "mfma_tile.hpp"

namespace gcp {

hipError_t dense_mfma_launch_poisson_id(const DenseCall& c, const MfmaPlan& p, float* G1p, float* G2p, float* G3p,
                                   float* gsp, float* lossp) {
  return by_rank<kPoissonId>(c, p, G1p, G2p, G3p, gsp, lossp);
}

}  // namespace gcp
