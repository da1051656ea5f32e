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
};
struct DivArgs {
  const double *in, *d;              // [n]
  double *out;                       // [n]; out[j] = in[j] / d[j] (in[j] where d[j] <= 0)
  int64_t n;
};
const void *divide_kernel();
const void *mdot_part_kernel();
const void *mdot_final_kernel();
const void *lincomb_kernel();
int lm_threads();

}  // namespace sr
