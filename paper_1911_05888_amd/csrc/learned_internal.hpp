// Learned post-smoothing correction: device parameter layout and launchers.
//
// Network of one finest-level element E (3^d patch of elements around it):
//   a1 = W1 z + b1 (H = 16), h1 = relu(a1), a2 = W2 h1 + b2, h2 = relu(a2),
//   y = W3 h2 + b3 (n_b outputs), dx_E = y * s_f * c_f per field f.
// z holds, per patch element F (offsets in {-1,0,1}^d, axis 0 fastest), the
// n_b residual coefficients of F divided by the global RMS s_f of their field
// (velocity or pressure) and log10 of F's mean viscosity.
//
// Device layout (padded so that every 8-entry group of the first layer lies
// in one patch element and every matrix dimension is a multiple of 16):
//   CHP  = roundup(n_b + 1, 8) channels per patch element (zeros beyond n_b)
//   K1P  = roundup(3^d * CHP, 32) first-layer inputs
//   NOUT = roundup(n_b, 16) outputs
//   params (FP32 master, and a BF16 copy of the weight matrices at the same
//   offsets): W1 [H][K1P] | b1 [H] | W2 [H][H] | b2 [H] | W3 [NOUT][H] | b3 [NOUT]
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/ldgs.h"

namespace ldgs {

constexpr int NET_H = 16;

struct NetShape {
  int d, p, nb, nq, ch, chp, noff, k1, k1p, nout;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, total;   // offsets into the padded parameter vector
  int64_t flat_total;                              // unpadded host layout size
};
NetShape net_shape(int d, int p);

// device parameter pointers
struct NetDev {
  const float* master;      // padded FP32
  const uint16_t* wbf;      // padded BF16 copy (weight segments)
};

// sums of squares of the velocity and pressure coefficients of r (unscaled by
// dscale when given) into sums[2] (device, FP64); part: nblk*2 doubles scratch
template <typename T>
int launch_field_sumsq(void* stream, int64_t ne, int nb, int nvel, const T* r, const double* dscale,
                       double* part, int nblk, double* sums);

// out = base + dx (base may be null), dx from residual r (FP32 or FP64,
// divided by dscale when given), scales from sums (device), per-element
// log10 mean viscosity logmu (device FP32)
template <typename Tin>
int launch_net_apply(void* stream, int d, int p, int n, int lgn, int permask, const Tin* r, const double* dscale,
                     const float* logmu, const double* sums, double cnt_u, double cnt_p, double c_u, double c_p,
                     NetDev net, const double* base, double* out);

// minimal-residual step of the correction: sums[0] = r . q, sums[1] = q . q
// (FP64 accumulation; part: nblk*2 doubles scratch); then
// out = base + w dx with w = sums[0] / sums[1] (0 if sums[1] = 0), w stored
// in sums[2] (sums: 3 device doubles); sums null: the full step w = 1
template <typename T>
int launch_minres_sums(void* stream, int64_t n, const T* r, const T* q, double* part, int nblk, double* sums);
int launch_minres_update(void* stream, int64_t n, double* sums, const double* base, const double* dx, double* out);

// crops for training: features [(C+2)^d][CHP] BF16 of r / s (and log10 mu),
// targets [C^d][n_b] BF16 of e / s, for ncrop crops with the given origins
// (device int [ncrop][d]); element fields r, e FP64 on the n^d grid
int launch_collect_crops(void* stream, int d, int p, int n, int lgn, int permask, int C, int lgC, int ncrop,
                         const int* origins, const double* r, const double* e, const float* logmu,
                         const double* sums, double cnt_u, double cnt_p, uint16_t* feat, uint16_t* targ);

// one forward/backward pass over the crops listed in batch (device int
// [nbatch]); gradients (padded layout, FP32) and the summed squared error are
// accumulated into grad and loss
int launch_train_grad(void* stream, int d, int p, int C, int lgC, int nbatch, const int* batch,
                      const uint16_t* feat, const uint16_t* targ, double c_u, double c_p, double inv_count,
                      NetDev net, float* grad, double* loss);

// Adam step on the padded parameter vector; refreshes the BF16 copy
int launch_adam(void* stream, int64_t n, float* master, uint16_t* wbf, const float* grad, float* m, float* v,
                float lr, float beta1, float beta2, float eps, float bc1, float bc2);

int launch_to_bf16(void* stream, int64_t n, const float* src, uint16_t* dst);

// Device address, on the current GPU, of the fixed training workspace of
// LDGS_TRAIN_WORKSPACE_BYTES (looked up once per GPU); 0 on success.
int train_workspace(void** ptr);

}  // namespace ldgs
