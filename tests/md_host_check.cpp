// Host build of the multiple-double header: 1/sqrt and reciprocals by the
// full and the shortened precision-doubling sequences on seeded inputs, and
// (argument "add") the accurate addition and subtraction of operands read
// from stdin; every limb printed exactly (hex floats) for an exact rational
// check in Python.
#include "../paper_2301_12659_amd/csrc/md.hpp"
#include <cstdio>
#include <random>
#include <string>

template <int L> void run(std::mt19937_64 &g, int count) {
  std::uniform_real_distribution<double> u(0.5, 2.0), s(-1.0, 1.0);
  for (int t = 0; t < count; ++t) {
    double a[L];
    a[0] = u(g) * std::ldexp(1.0, (int)(s(g) * 20));
    for (int l = 1; l < L; ++l) a[l] = a[l - 1] * std::ldexp(s(g), -53);  // nonoverlapping limbs
    double y[L], r[L], y2[L], r2[L];
    md::rsqrt_short<L>(a, y);
    md::recip_short<L>(a, r);
    md::rsqrt_newton<L>(a, y2);
    md::recip_newton<L>(a, r2);
    printf("%d", L);
    for (double *v : {a, y, r, y2, r2})
      for (int l = 0; l < L; ++l) printf(" %a", v[l]);
    printf("\n");
  }
}

// a + b and a - b by the accurate routines for operands read from stdin
// (lines "L a_0 .. a_{L-1} b_0 .. b_{L-1}" in hex floats).
template <int L> void add_case() {
  double a[L], b[L], s[L], d[L];
  for (int l = 0; l < L; ++l)
    if (scanf("%la", &a[l]) != 1) return;
  for (int l = 0; l < L; ++l)
    if (scanf("%la", &b[l]) != 1) return;
  md::MD<L>::add_acc(a, b, s);
  md::MD<L>::sub_acc(a, b, d);
  printf("%d", L);
  for (double *v : {s, d})
    for (int l = 0; l < L; ++l) printf(" %a", v[l]);
  printf("\n");
}

int main(int argc, char **argv) {
  if (argc > 1 && std::string(argv[1]) == "add") {
    int L;
    while (scanf("%d", &L) == 1) {
      if (L == 2) add_case<2>();
      else if (L == 4) add_case<4>();
      else if (L == 8) add_case<8>();
      else return 1;
    }
    return 0;
  }
  std::mt19937_64 g(3);
  run<2>(g, 200);
  run<4>(g, 200);
  run<8>(g, 200);
  return 0;
}
