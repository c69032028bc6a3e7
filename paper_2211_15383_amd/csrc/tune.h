// Launch-variant autotuner (tune.hip).
#pragma once

#include "common.h"

// Times every launch variant of the tuned kernels on each level of H at nrhs right-hand
// sides (reps launches per variant) and keeps the fastest in H->lv[].kv; picks / best_us /
// default_us (nullable, [levels][KV_COUNT]) receive the chosen value (-1: kernel not run
// on that level), its time and the built-in rule's time per launch (0 for cached choices).
void tune_kernels(dmlmc_hier* H, int nrhs, int reps, const char* cache_path, int* picks, double* best_us,
                  double* default_us);
void set_kernel_variant(dmlmc_hier* H, int level, int kernel, int value);
// the matrix-core transfer kernels handle this level's interpolation (stencil.hip)
bool transfer16_available(const Level& L);
bool transfer16_pair_available(const Level& L);
// whether the launch rules of a level currently select the pair-staged transfer kernels
// (which have no tile-count variants)
bool restrict16_pair_selected(const Level& L);
bool prolong16_pair_selected(const Level& L);
