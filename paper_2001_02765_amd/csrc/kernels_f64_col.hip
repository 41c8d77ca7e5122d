// Column kernels instantiated for double plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_col<double>(const Pack<ColArgs<double>> &, int, int, int, int, int, int,
                                    const C<double> *, const C<double> *, hipStream_t, int);

}  // namespace grav
