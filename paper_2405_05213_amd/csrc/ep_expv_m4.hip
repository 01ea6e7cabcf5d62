// Instantiations of the persistent projection kernel with the operator of the fourth-order
// scheme (Krylov-vector slices in LDS; FP64 and FP32 element kernels); a separate
// translation unit so that it compiles in parallel with the others.
#include "ep_expv.hpp"

namespace ep {

const void* expv_kernel_m4(int prec, int model, int ortho) {
  if (prec == 0) {
    if (model == kLinear) return expv_fn_m4<double, kLinear>(ortho);
    if (model == kNH) return expv_fn_m4<double, kNH>(ortho);
    if (model == kSVK) return expv_fn_m4<double, kSVK>(ortho);
    return expv_fn_m4<double, kYeoh>(ortho);
  }
  if (model == kLinear) return expv_fn_m4<float, kLinear>(ortho);
  if (model == kNH) return expv_fn_m4<float, kNH>(ortho);
  if (model == kSVK) return expv_fn_m4<float, kSVK>(ortho);
  return expv_fn_m4<float, kYeoh>(ortho);
}

}  // namespace ep
