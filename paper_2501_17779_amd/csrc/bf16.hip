// Split-BF16 dense-DFT path (placeholder translation unit; kernels follow).
#include "common.hpp"
