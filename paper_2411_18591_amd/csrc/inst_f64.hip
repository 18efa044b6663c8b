// Propagation kernels instantiated for complex128 fields.
#include "launch_impl.hpp"

namespace toprop {
template struct Launch<double>;
}  // namespace toprop
