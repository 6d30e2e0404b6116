// The RK stage kernel in the FP32-storage form (FP32 stage states, metrics
// and fluxes; FP64 Q^(0) and stage accumulation).  The kernel template is in
// fused_stage.hpp; this translation unit keeps the default instruction
// scheduling, under which the FP32 kernel fits four waves per SIMD without
// spilling.
#include "fused_stage.hpp"

namespace lesjet {

template int fused_chunk<float>(const Grid&, int);
template hipError_t launch_fused<float>(const float*, const float*, const Grid&, const Phys<float>&,
                                        int, int, float*, const double*, double*, double,
                                        const double*, const Phys<double>&, unsigned long long*,
                                        int, float*, const double*, hipStream_t);

}  // namespace lesjet
