// Host build of the per-structure superposition math (pcv_math.h) for CPU
// unit tests: the same functions the kernels inline, exposed with a C ABI.
#include <hip/hip_runtime.h>

#include "pcv_math.h"

extern "C" {

// Top eigenpair and rotation from a correlation matrix M (row-major 3x3).
// Returns 1 if the Jacobi fallback was used.
int pcvt_superpose(const double* M, double lam_up, double* lam, double* q, double* R, double* F) {
  double Fl[10];
  const int fb = pcv::top_eigenpair(M, lam_up, Fl, *lam, q);
  pcv::quat_to_rot(q, R);
  for (int k = 0; k < 10; ++k) F[k] = Fl[k];
  return fb;
}

void pcvt_char_poly(const double* M, double* c) {
  double F[10];
  pcv::horn_matrix(M, F);
  pcv::char_poly(M, F, c[0], c[1], c[2]);
}

double pcvt_jacobi_top(const double* M, double* q) {
  double F[10];
  pcv::horn_matrix(M, F);
  return pcv::jacobi_top(F, q);
}

void pcvt_rotation_adjoint(const double* F, double lam, const double* q, const double* G, double* Gamma) {
  pcv::rotation_adjoint(F, lam, q, G, Gamma);
}

}
