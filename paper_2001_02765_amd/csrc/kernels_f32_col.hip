// Column kernels instantiated for float plans.
#include "kernels_impl.hpp"

namespace grav {

template hipError_t launch_col<float>(const Pack<ColArgs<float>> &, int, int, int, int, int, int,
                                    const C<float> *, const C<float> *, hipStream_t, int);

}  // namespace grav
