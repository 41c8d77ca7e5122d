// Row kernels instantiated for float plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_row_fwd<float>(const Pack<RowFwdArgs<float>> &, int, int, int, bool, int64_t, int,
                                        const C<float> *, hipStream_t);
template hipError_t launch_row_inv<float>(const Pack<RowInvArgs<float>> &, int, int, int, int64_t, int,
                                        const C<float> *, hipStream_t);

}  // namespace grav
