// Job-queue passes instantiated for complex64 fields.
#include "queue_impl.hpp"

namespace toprop {
template struct QueueLaunch<float>;
}  // namespace toprop
