// Solve-path kernels instantiated for double plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_row_fwd<double>(const RowFwdArgs<double> &, int, int, bool, int, int,
                                        const C<double> *, hipStream_t);
template hipError_t launch_col<double>(const ColArgs<double> &, int, int, int, int, const C<double> *,
                                    const C<double> *, hipStream_t);
template hipError_t launch_row_inv<double>(const RowInvArgs<double> &, int, int, int, int,
                                        const C<double> *, hipStream_t);

}  // namespace grav
