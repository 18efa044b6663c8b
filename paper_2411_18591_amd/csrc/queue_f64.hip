// Job-queue passes instantiated for complex128 fields.
#include "queue_impl.hpp"

namespace toprop {
template struct QueueLaunch<double>;
}  // namespace toprop
