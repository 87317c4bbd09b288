// array_f64.hip -- array-section reduction kernels for f64 inputs.
#include "array_kernel.h"

namespace omprt {

ArrayLauncher array_launcher_f64(int op, bool vec, int u) {
    return array_launcher_impl<DT_F64>(op, vec, u);
}

}  // namespace omprt
