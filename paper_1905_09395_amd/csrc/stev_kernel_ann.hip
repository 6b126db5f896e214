// Instantiations of the persistent STEV kernel with the paper's sigmoid
// thermo network (Sec 3) in FP64 and FP32, one per compiled variant shape.
#include "stev_persistent.h"
#include "stev_variants.h"

namespace stev {

#define STEV_INST_ANN(R, G, RPL, RRPL, SPL, CSRR) \
  reinterpret_cast<const void *>(&stev_persistent<R, G, RPL, RRPL, SPL, CSRR, kThAnn, false>)

const void *const kAnnVariants[][2] = {
#define STEV_VARIANT(G, RPL, RRPL, SPL, CSRR)              \
  {STEV_INST_ANN(double, G, RPL, RRPL, SPL, CSRR),         \
   STEV_INST_ANN(float, G, RPL, RRPL, SPL, CSRR)},
    STEV_VARIANT_LIST
#undef STEV_VARIANT
};

}  // namespace stev
