// Host-side dense helpers for the Rayleigh-Ritz steps (FP64).
#pragma once

#include <complex>
#include <vector>

int eigh_jacobi(int n, std::vector<std::complex<double>> A, std::vector<double>& w,
                std::vector<std::complex<double>>& Z);
int eigh_tridiag(int n, std::vector<std::complex<double>> A, std::vector<double>& w,
                 std::vector<std::complex<double>>& Z);
bool cholesky_lower(int n, std::vector<std::complex<double>>& A);
void lower_inverse(int n, std::vector<std::complex<double>>& Lm);
