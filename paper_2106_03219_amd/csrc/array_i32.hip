// array_i32.hip -- array-section reduction kernels for i32 inputs.
#include "array_kernel.h"

namespace omprt {

ArrayLauncher array_launcher_i32(int op, bool vec, int u) {
    return array_launcher_impl<DT_I32>(op, vec, u);
}

}  // namespace omprt
