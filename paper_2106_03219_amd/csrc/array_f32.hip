// array_f32.hip -- array-section reduction kernels for f32 inputs.
#include "array_kernel.h"

namespace omprt {

ArrayLauncher array_launcher_f32(int op, bool vec, int u) {
    return array_launcher_impl<DT_F32>(op, vec, u);
}

}  // namespace omprt
