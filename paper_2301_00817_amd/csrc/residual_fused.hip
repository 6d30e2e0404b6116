// The RK stage kernel in FP64 (plain form).  The kernel template is in
// fused_stage.hpp; each precision is its own translation unit so that each
// takes the instruction scheduling that measured faster for it (the build
// schedules this one for instruction-level parallelism).
#include "fused_stage.hpp"

namespace lesjet {

template int fused_chunk<double>(const Grid&, int);
template hipError_t launch_fused<double>(const double*, const double*, const Grid&,
                                         const Phys<double>&, int, int, double*, const double*,
                                         double*, double, const double*, const Phys<double>&,
                                         unsigned long long*, int, double*, const double*,
                                         hipStream_t);

}  // namespace lesjet
