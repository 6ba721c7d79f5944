// Operation count of the per-lane arithmetic of the HGKS kernels: the same
// templated functions the kernels run, instantiated on the host with a
// scalar type that counts every add/subtract, multiply, divide and
// transcendental (sqrt, exp, erfc) it performs.  A fused multiply-add in the
// generated code is two operations here (one multiply, one add).
//
// Prints one JSON object: operations per Gauss-point flux (box grid,
// viscous collision time, no fallback), per cell reconstruction of the five
// variables, and per cell stage update.
#include <cmath>
#include <cstdio>

#include "box_kernels.h"

namespace cnt {
long long add = 0, mul = 0, dv = 0, tr = 0;
void reset() { add = mul = dv = tr = 0; }
long long total() { return add + mul + dv + tr; }
}  // namespace cnt

struct Cnt {
  double v;
  HGKS_FN Cnt() : v(0.0) {}
  HGKS_FN Cnt(double x) : v(x) {}
  HGKS_FN Cnt(int x) : v((double)x) {}
};
inline Cnt operator+(Cnt a, Cnt b) { ++cnt::add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++cnt::add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++cnt::mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++cnt::dv; return Cnt(a.v / b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline Cnt exp(Cnt x) { ++cnt::tr; return Cnt(std::exp(x.v)); }
inline Cnt log(Cnt x) { ++cnt::tr; return Cnt(std::log(x.v)); }

namespace hgks {
template <> HGKS_FN Cnt d_exp<Cnt>(Cnt x) { ++cnt::tr; return Cnt(std::exp(x.v)); }
template <> HGKS_FN Cnt d_erfc<Cnt>(Cnt x) { ++cnt::tr; return Cnt(std::erfc(x.v)); }
template <> HGKS_FN Cnt d_sqrt<Cnt>(Cnt x) { ++cnt::tr; return Cnt(std::sqrt(x.v)); }
template <> HGKS_FN Cnt d_rcp<Cnt>(Cnt x) { ++cnt::dv; return Cnt(1.0 / x.v); }
}  // namespace hgks

using namespace hgks;

int main() {
  // A Taylor-Green-like interface state: rho ~ 1, p ~ 71.4, |U| ~ 1.
  GasParams<Cnt> g;
  const double K = (5.0 - 3.0 * 1.4) / 0.4;
  g.gm1 = Cnt(0.4); g.K = Cnt(K); g.K3 = Cnt(K + 3.0); g.K2 = Cnt(K + 2.0);
  g.inv_K3 = Cnt(1.0 / (K + 3.0)); g.two_gm1 = Cnt(2.0 / 0.4);
  g.mu = Cnt(1.0 / 1600.0); g.tau_eps = Cnt(0.01); g.tau_C = Cnt(1.0); g.viscous = 1;

  // Coefficients of two cells (5 variables x 10) in the kernel layout.
  const size_t NR = 2;
  static Cnt coef[coef_elems(NR, sizeof(Cnt))];
  const double base[5] = {1.0, 0.6, -0.4, 0.1, 178.9};
  for (int v = 0; v < 5; ++v)
    for (int k = 0; k < 10; ++k)
      for (size_t c = 0; c < NR; ++c)
        coef[coef_cell<Cnt>(c) + (v * 10 + k) * kCB<Cnt>] = Cnt(k == 0 ? base[v] : 0.01 * (k + v + c));
  const Cnt invd[3] = {Cnt(20.0), Cnt(20.0), Cnt(20.0)};

  cnt::reset();
  FluxAcc<Cnt> acc;
  {
    Cnt W[5], dW[3][5];
    eval_box_gp<0>(coef, 0, Cnt(0.5), Cnt(0.2887), Cnt(-0.2887), false, invd, W, dW);
    side_terms<+1, false, true>(W, dW, g, acc);
  }
  {
    Cnt W[5], dW[3][5];
    eval_box_gp<0>(coef, 1, Cnt(-0.5), Cnt(0.2887), Cnt(-0.2887), false, invd, W, dW);
    side_terms<-1>(W, dW, g, acc);
  }
  Cnt F[5], dF[5];
  finish_flux(acc, g, Cnt(1.5e-3), Cnt(1.0 / 1.5e-3), F, dF);
  // Face weight and the four-point face sum: 10 products per point and
  // 3 additions per face and value (7.5 per point).
  const double flux_gp = (double)cnt::total() + 10.0 + 7.5;
  const long long f_add = cnt::add, f_mul = cnt::mul, f_div = cnt::dv, f_tr = cnt::tr;

  // The same with the Prandtl correction (Pr 0.72, constant mu): the
  // instantiation the Taylor-Green benchmark runs.
  g.pr_fix = Cnt(1.0 / 0.72 - 1.0);
  cnt::reset();
  {
    FluxAcc<Cnt> accp;
    {
      Cnt W[5], dW[3][5];
      eval_box_gp<0>(coef, 0, Cnt(0.5), Cnt(0.2887), Cnt(-0.2887), false, invd, W, dW);
      side_terms<+1, true, true>(W, dW, g, accp);
    }
    {
      Cnt W[5], dW[3][5];
      eval_box_gp<0>(coef, 1, Cnt(-0.5), Cnt(0.2887), Cnt(-0.2887), false, invd, W, dW);
      side_terms<-1, true>(W, dW, g, accp);
    }
    finish_flux<true>(accp, g, Cnt(1.5e-3), Cnt(1.0 / 1.5e-3), F, dF);
  }
  const double flux_gp_pr = (double)cnt::total() + 10.0 + 7.5;

  // Reconstruction of one cell: differences (double), five variables, and
  // the sufficient positivity test (about 20 operations).
  WenoParams<Cnt> P;
  P.gamma0 = Cnt(0.94); P.Gamma = Cnt(0.0025); P.eps = Cnt(1e-8);
  for (int d = 0; d < 3; ++d) { P.kl[d] = Cnt(1.0); P.kq[d] = Cnt(13.0 / 3.0); P.km[d] = Cnt(7.0 / 6.0); }
  cnt::reset();
  for (int v = 0; v < 5; ++v) {
    Cnt d[27];
    for (int i = 0; i < 27; ++i) d[i] = Cnt(0.001 * (i % 7) - 0.002);
    BoxRecon<Cnt> r;
    weno_box(d, P, r);
  }
  const double recon_cell = (double)cnt::total() + 5 * 18 + 20;
  const long long r_div = cnt::dv;

  // Stage update of one cell: 6 face differences of 10 values, then per
  // variable L, dL (2 products) and the stage formulas (at most 8).
  const double update_cell = 60 + 5 * (2 + 8);

  std::printf(
      "{\"flux_gp_ops\": %.1f, \"flux_gp_add\": %lld, \"flux_gp_mul\": %lld, \"flux_gp_div\": %lld, "
      "\"flux_gp_transcendental\": %lld, \"recon_cell_ops\": %.1f, \"recon_cell_div\": %lld, "
      "\"update_cell_ops\": %.1f, \"gp_per_cell_stage\": 12, \"flux_gp_ops_prandtl\": %.1f}\n",
      flux_gp, f_add, f_mul, f_div, f_tr, recon_cell, r_div, update_cell, flux_gp_pr);
  return 0;
}
