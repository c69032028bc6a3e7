// Direct coarsest solve by the explicit inverse (complex FP32, matrix cores).
#pragma once

#include "common.h"

// Computes D_L^-1 column by column (multi-RHS solves, the coarsest deflation defl in the
// V-cycles if given) into H->coarse_dinv.
void build_coarse_direct(dmlmc_hier* H, const dmlmc_defl* defl);
// Y = D_L^-1 B for nrhs complex-FP32 vectors [nrhs][n_L].
void apply_coarse_direct(dmlmc_hier* H, const c64* B, c64* Y, int nrhs);
