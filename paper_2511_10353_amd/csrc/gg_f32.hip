// Single-precision instantiation of the kernels and launchers.
#include "ops_impl.h"

namespace gg {
template struct Ops<float>;
}  // namespace gg
