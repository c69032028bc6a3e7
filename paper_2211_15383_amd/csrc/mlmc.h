// Internal MLMC driver interface.
#pragma once

#include "common.h"

void run_mlmc(dmlmc_hier* H, const dmlmc_defl* defl, const dmlmc_mlmc_params* p, dmlmc_trace_result* res);
