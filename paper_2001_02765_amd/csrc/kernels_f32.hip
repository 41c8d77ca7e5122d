// Solve-path kernels instantiated for float plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_row_fwd<float>(const RowFwdArgs<float> &, int, int, bool, int, int,
                                        const C<float> *, hipStream_t);
template hipError_t launch_col<float>(const ColArgs<float> &, int, int, int, int, const C<float> *,
                                    const C<float> *, hipStream_t);
template hipError_t launch_row_inv<float>(const RowInvArgs<float> &, int, int, int, int,
                                        const C<float> *, hipStream_t);

}  // namespace grav
