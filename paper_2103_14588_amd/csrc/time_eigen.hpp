// time_eigen.hpp -- generalised eigen-decomposition of the Galerkin time
// pencil (host code; definitions and method in time_eigen.hip).
#pragma once

#include <complex>
#include <vector>

namespace dst {

constexpr int kTimeEigenMax = 2048;

// D W = M W diag(lam) for the n x n time factors with step h; W and
// Q = W^{-1} M^{-1} row-major.  Returns 0, or an error code with the message set.
int time_eigen(int n, double h, std::vector<std::complex<double>> &lam,
               std::vector<std::complex<double>> &W, std::vector<std::complex<double>> &Q);

}  // namespace dst
