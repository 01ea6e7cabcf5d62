// Instantiations of the persistent projection kernel with the Krylov-vector slices in
// device memory (meshes whose slices do not fit in LDS on one workgroup per CU); a
// separate translation unit so that the two sets compile in parallel.
#include "ep_expv.hpp"

namespace ep {

const void* expv_kernel_global(int prec, int model, int ortho) { return expv_kernel_sg<1>(prec, model, ortho); }

}  // namespace ep
