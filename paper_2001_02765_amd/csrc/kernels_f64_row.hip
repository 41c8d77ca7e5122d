// Row kernels instantiated for double plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_row_fwd<double>(const Pack<RowFwdArgs<double>> &, int, int, int, bool, int64_t, int,
                                        const C<double> *, hipStream_t);
template hipError_t launch_row_inv<double>(const Pack<RowInvArgs<double>> &, int, int, int, int64_t, int,
                                        const C<double> *, hipStream_t);

}  // namespace grav
