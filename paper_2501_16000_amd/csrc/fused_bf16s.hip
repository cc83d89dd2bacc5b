// fused_bf16s.hip -- the fused multi-step sweeps (lb_step and the server) for
// shifted BF16 storage: instantiations of fused_impl.hpp.
#include "fused_impl.hpp"

namespace oreg {

template hipError_t fused_launch_st<LB_BF16S>(int, int, int, const void*, void*, const Geometry&,
                                           const Coef64&, int, int, hipStream_t);
template hipError_t fused_occupancy_st<LB_BF16S>(int, int*);
template hipError_t batched_fused_launch_st<LB_BF16S>(int, const LatticeDesc*, const int*, int64_t,
                                                   int64_t, hipStream_t);

}  // namespace oreg
