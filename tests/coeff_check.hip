// Host check of the cumulant's linear form (built and run by
// tests/test_cumulant_linear_form.py; no GPU needed).  Each input line holds a
// convention (0 click, 1 parity), NB = |B|, the B-only correlators m(U) for
// every U subset of B (bit j <-> b_j, m(empty) = 1) and the vacuum
// probabilities p({a} + V) for every V subset of B; the program prints the
// correlator and cumulant of S = {a} + B that the kernels form from them:
// m(S) from nu(B) = sum_V s(V) p({a} + V), and k(S) = sum_V c_B(V) p({a} + V)
// with the coefficients of cumulant_coefficients (gbs_subset.h).
#include <cstdio>

#include "gbs_subset.h"

using namespace gbs;

template <int NB, int CONV>
static void eval(const double* mu, const double* pa) {
  constexpr int NU = 1 << NB;
  double m[NU], c[NU];
  for (int u = 0; u < NU; ++u) m[u] = mu[u];
  cumulant_coefficients<NB, CONV>(m, c);
  double nu = 0.0, k = 0.0;
  for (int v = 0; v < NU; ++v) {
    nu = fma(vacuum_sign<CONV>(v), pa[v], nu);
    k = fma(c[v], pa[v], k);
  }
  const double mS = (CONV == GBS_CLICK) ? m[NU - 1] - nu : fma((NB & 1) ? -2.0 : 2.0, nu, -m[NU - 1]);
  printf("%.17g %.17g\n", mS, k);
}

template <int CONV>
static void dispatch(int nb, const double* mu, const double* pa) {
  switch (nb) {
    case 1: eval<1, CONV>(mu, pa); break;
    case 2: eval<2, CONV>(mu, pa); break;
    case 3: eval<3, CONV>(mu, pa); break;
    case 4: eval<4, CONV>(mu, pa); break;
    default: printf("nan nan\n");
  }
}

int main() {
  int conv, nb;
  while (scanf("%d %d", &conv, &nb) == 2) {
    if (nb < 1 || nb > 4) return 2;
    double mu[16], pa[16];
    for (int i = 0; i < (1 << nb); ++i)
      if (scanf("%lf", &mu[i]) != 1) return 3;
    for (int i = 0; i < (1 << nb); ++i)
      if (scanf("%lf", &pa[i]) != 1) return 3;
    if (conv) dispatch<GBS_PARITY>(nb, mu, pa);
    else dispatch<GBS_CLICK>(nb, mu, pa);
  }
  return 0;
}
