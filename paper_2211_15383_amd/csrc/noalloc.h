// Allocation-free deflation projection (noalloc.hip).
#pragma once

#include "common.h"

// Size of the per-device scratch array in bytes.
size_t noalloc_scratch_bytes();
// Device address of the scratch array on the current device (hipGetSymbolAddress).
void* noalloc_scratch_address();
// out = in - W (W^H in) with the deflation's FP32 matrix-core kernels, partials in the
// context's scratch address; validates the scratch size, synchronises the stream.
void deflate_project_noalloc(dmlmc_ctx* ctx, const dmlmc_defl* D, const void* in, void* out, int nrhs);
