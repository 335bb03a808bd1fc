// Block Arnoldi and Lanczos steps for block size s = 8 (FP64 and FP32 bases).
#include "arnoldi_impl.h"

ARN_UNIT(8)
