// Host driver for the sanitizer build of the superposition math
// (pcv_hosttest.cpp): random and degenerate correlation matrices through the
// eigen-solve, the Jacobi fallback and the rotation adjoint; exits non-zero
// on a non-finite result.  Built and run by tests/test_library_cpu.py with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code.
#include <cmath>
#include <cstdio>
#include <random>

extern "C" {
int pcvt_superpose(const double* M, double lam_up, double* lam, double* q, double* R, double* F);
void pcvt_char_poly(const double* M, double* c);
double pcvt_jacobi_top(const double* M, double* q);
void pcvt_rotation_adjoint(const double* F, double lam, const double* q, const double* G, double* Gamma);
}

int main() {
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  int bad = 0;
  for (int t = 0; t < 2000; ++t) {
    double M[9], G[9];
    for (int k = 0; k < 9; ++k) {
      M[k] = nd(rng);
      G[k] = nd(rng);
    }
    if (t % 7 == 0)   // rank-deficient: a degenerate spectrum (Jacobi fallback)
      for (int k = 0; k < 3; ++k) M[6 + k] = 0.0;
    if (t % 11 == 0)
      for (int k = 0; k < 9; ++k) M[k] = 0.0;
    double nrm = 0.0;
    for (int k = 0; k < 9; ++k) nrm += M[k] * M[k];
    double lam, q[4], R[9], F[10], c[3], Gam[9], qj[4];
    pcvt_superpose(M, std::sqrt(3.0 * nrm) + 1.0, &lam, q, R, F);
    pcvt_char_poly(M, c);
    const double lj = pcvt_jacobi_top(M, qj);
    pcvt_rotation_adjoint(F, lam, q, G, Gam);
    double s = lam + lj + c[0] + c[1] + c[2];
    for (int k = 0; k < 9; ++k) s += R[k] + Gam[k];
    if (!std::isfinite(s)) ++bad;
  }
  std::printf("sanitized host math: %d non-finite results\n", bad);
  return bad == 0 ? 0 : 1;
}
