// Internal hierarchy-construction interfaces.
#pragma once

#include "common.h"

void upload_links(dmlmc_ctx* ctx, Level& L, const double* theta_host, int antiperiodic);
void build_interpolator(dmlmc_ctx* ctx, Level& L, const c128* V, int N);
Level galerkin_level(dmlmc_ctx* ctx, const Level& F);
void orthonormalise(dmlmc_hier* H, c128* V, int N, int64_t n);
// Builds levels 2..L of H (H->lv holds level 1 and H->plan the coarsening steps);
// import_tv[l-1], when non-null, are host test vectors for step l.
void build_levels(dmlmc_hier* H, const std::vector<const c128*>& import_tv);
