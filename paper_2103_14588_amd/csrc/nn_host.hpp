// nn_host.hpp -- host-side interface of the network shared by the solver.
#pragma once

#include <cstddef>

#include "common.hpp"

namespace dst {

constexpr int kWgradBlocks = 512;  // workgroups (and partial rows) of the weight gradient
constexpr int kBiasBlocks = 256;
constexpr int kLossBlocks = 256;

// byte offsets inside a network workspace
struct NnLayout {
  size_t a0, a1, a2, a3, out;              // activations (bf16) and output (FP32)
  size_t g4, g3, g2, g1;                   // back-propagated gradients (bf16), training only
  size_t wpart, bpart, lpart, grad, loss;  // partial sums, parameter gradient, loss
  size_t total;
};

NnLayout nn_layout(int nt, int ny, int nx, bool training);

// z (+)= out_scale * N(in_scale * v) for a 2+1D field [nt][ny][nx][2] complex
// of precision prec (64: complex128, 32: complex64).
int nn_apply_add(const dirac_st_nn *net, int nt, int ny, int nx, const void *v, int prec,
                 double in_scale, double out_scale, void *z, int accumulate, unsigned char *work,
                 hipStream_t s);

}  // namespace dst
