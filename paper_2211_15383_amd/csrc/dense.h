// Direct coarsest solve by the explicit inverse (complex FP32 or FP16, matrix cores).
#pragma once

#include "common.h"

// Computes D_L^-1 column by column (multi-RHS solves, the coarsest deflation defl in the
// V-cycles if given) into H->coarse_dinv.
void build_coarse_direct(dmlmc_hier* H, const dmlmc_defl* defl, double rtol);
// Rounds the FP32 inverse to complex FP16 (one power-of-two scale) into H->coarse_dinv16.
void build_coarse_direct16(dmlmc_hier* H);
// Rounds the FP32 inverse to 8-bit floats (sign, 4 exponent bits with bias 7, 3 mantissa
// bits; each row scaled by a power of two below 256) into H->coarse_dinv8, the row
// factors into H->coarse_dinv8_rows.
void build_coarse_direct8(dmlmc_hier* H);
// Y = D_L^-1 B for nrhs complex-FP32 vectors [nrhs][n_L] with the inverse of
// H->coarse_direct_mode (1: FP32, 2: FP16, 3: 8-bit).
void apply_coarse_direct(dmlmc_hier* H, const c64* B, c64* Y, int nrhs);
