// ops.h -- element types and reduction operators, as numbered in the C ABI
// (omprt_dtype, omprt_op), shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>

namespace omprt {

enum { DT_I32 = 0, DT_I64 = 1, DT_F32 = 2, DT_F64 = 3, DT_BF16 = 4, DT_COUNT = 5 };

// The reduction identifiers of the OpenMP reduction clause: + max min on
// every type, * on every type, & | ^ on integers, && || on every type.
enum {
    OP_SUM = 0, OP_MAX = 1, OP_MIN = 2, OP_PROD = 3, OP_BAND = 4, OP_BOR = 5, OP_BXOR = 6,
    OP_LAND = 7, OP_LOR = 8, OP_COUNT = 9
};
// True when (dtype, op) is a reduction the library implements.
__host__ __device__ constexpr bool op_defined(int dt, int op) {
    return op >= 0 && op < OP_COUNT && dt >= 0 && dt < DT_COUNT &&
           !((op == OP_BAND || op == OP_BOR || op == OP_BXOR) && dt != DT_I32 && dt != DT_I64);
}

}  // namespace omprt
