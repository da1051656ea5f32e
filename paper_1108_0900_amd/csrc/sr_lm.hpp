// Argument blocks of the vector kernels of the generalized Davidson solver.
#pragma once
#include "sr_launch.hpp"

namespace sr {

// Generalized Davidson of the linear method: subspace dot products and combinations.
constexpr int kLmMaxSub = 64;        // largest subspace
struct MdotArgs {
  const double *X;                   // [m][ld]
  int64_t ld, n;
  int m, nb;                         // rows of X; workgroups of the partial pass
  const double *w;                   // [n]
  double *part;                      // [nb][m]
  double *out;                       // [m]
};
struct LincombArgs {
  const double *X, *Z;               // [mx][ld], [mz][ld]
  int mx, mz;
  int64_t ld, n;
  double beta;
  double *out;                       // [n]
  double ca[kLmMaxSub], cz[kLmMaxSub];
  const double *cdev;                // or nullptr: X's coefficients are cdev_sign * cdev[i]
  double cdev_sign;                  // (device memory, written by an earlier kernel)
  const double *bdev;                // or nullptr: beta = 1 / sqrt(*bdev) (device memory)
};
struct DivArgs {
  const double *in;                  // [n]
  const double *dh, *ds;             // [n] diag H (or nullptr) and diag S
  double *out;                       // [n]; out[j] = in[j] / (dh[j] - theta ds[j]), or in[j] / ds[j]
  int64_t n;
  double theta;
};
const void *divide_kernel();
// diag H of the linear method, H_jj = (1/N) sum_k Oc_kj (E_k Oc_kj + D_kj), j < n_p
struct DiagHArgs {
  Operand o, d;                      // O and D (single code plane each)
  const double *mean;                // [n_p] column means of O
  const double *E;                   // [n_s]
  int64_t n_s, n_p, rs;              // rows per split
  int SP;                            // splits (grid y)
  double *part;                      // [SP][n_p]
  double *out;                       // [n_p]
};
const void *diagh_part_kernel(int dt);
const void *diagh_final_kernel();
const void *mdot_part_kernel();
const void *mdot_final_kernel();
const void *lincomb_kernel();
int lm_threads();

}  // namespace sr
