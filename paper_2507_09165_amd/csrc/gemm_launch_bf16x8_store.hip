// Instantiation of the symmetric GEMM kernels for bf16x8 work matrices with the
// store epilogue (see gemm_sym_kernel.hpp).
#include "gemm_sym_kernel.hpp"

namespace psd {
template hipError_t gemm_launch_part<DT_BF16X8, EPI_STORE>(const GemmArgs &, bool, bool, int, int64_t, hipStream_t, int);
}  // namespace psd
