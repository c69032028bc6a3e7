// Tall-skinny FP64 block products (device operands, [count][n] complex128).
#pragma once

#include "common.h"

// G[r * na + i] = <A_i, B_r> for i < na, r < nb (device G); scratch holds partial sums.
void ts_gram(dmlmc_ctx* ctx, const c128* A, int na, const c128* B, int nb, int64_t n, c128* G, DevBuf& scratch);
// out_r = sum_i S[r * ny + i] Y_i for r < nr (device S); out must not alias Y.
void ts_rotate(dmlmc_ctx* ctx, const c128* Y, int ny, const c128* S, int nr, int64_t n, c128* out);
