// Internal MLMC driver interface.
#pragma once

#include "common.h"

void run_mlmc(dmlmc_hier* H, const dmlmc_defl* defl, const dmlmc_mlmc_params* p, dmlmc_trace_result* res);
// Deflated plain Hutchinson at the fine level (result index 0).
void run_hutchinson(dmlmc_hier* H, const dmlmc_defl* fine, const dmlmc_defl* coarsest, const dmlmc_mlmc_params* p,
                    dmlmc_trace_result* res);
// Times one block of samples per level for each candidate block size; returns the best.
int tune_rhs_block(dmlmc_hier* H, const dmlmc_defl* defl, const int* cand, int ncand, dmlmc_precision prec,
                   double rtol, uint64_t noise_seed, double* sec_per_sample);
