// array_bf16.hip -- array-section reduction kernels for bf16 inputs.
#include "array_kernel.h"

namespace omprt {

ArrayLauncher array_launcher_bf16(int op, bool vec, int u) {
    return array_launcher_impl<DT_BF16>(op, vec, u);
}

}  // namespace omprt
