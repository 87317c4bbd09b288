// array_i64.hip -- array-section reduction kernels for i64 inputs.
#include "array_kernel.h"

namespace omprt {

ArrayLauncher array_launcher_i64(int op, bool vec, int u) {
    return array_launcher_impl<DT_I64>(op, vec, u);
}

}  // namespace omprt
