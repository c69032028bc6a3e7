// Dense Hermitian eigensolver on the device (jacobi.hip).
#pragma once

#include <vector>

#include "common.h"

struct JacobiResult {
  int sweeps = 0;
  double offmax = 0.0;  // largest relative off-diagonal entry met in the last sweep
  bool converged = false;
};

// A: device, order n, column-major (A(i, j) at j * n + i), Hermitian up to rounding (its
// Hermitian part is used); not modified.
// On return w (host) holds the eigenvalues ascending and S (device, n x n column-major)
// the eigenvectors as columns in the same order.  work: device scratch, grown as needed
// (about 32 n^2 bytes).  Sweeps stop when the largest |M_pq| / sqrt(|M_pp M_qq|) met in a
// sweep is <= tol, or after max_sweeps.
JacobiResult jacobi_eigh(dmlmc_ctx* ctx, const c128* A, int n, c128* S, std::vector<double>& w, DevBuf& work,
                         double tol = 1e-12, int max_sweeps = 40);
