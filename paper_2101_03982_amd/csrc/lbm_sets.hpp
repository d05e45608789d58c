// Velocity sets of the semi-Lagrangian lattice Boltzmann library, as
// compile-time tables.
//
// Values are the ones printed in the paper (Wilde et al., "Cubature rules for
// weakly and fully compressible off-lattice Boltzmann methods"): Tables
// tab:d3q13 and tab:d3q21, App. C (D2Q19), App. D (D3V27, rows marked "(cyc)"
// stand for their cyclic shifts), App. E (D3Q45); the Gauss-Hermite product
// sets of Sec. 1 (D2Q9 and D3Q27 from D1Q3, D2Q25 from the degree-nine D1Q5
// whose nodes are the roots 0, +-sqrt(5 -+ sqrt 10) of He_5 and whose weights
// are 8/15 and (7 +- 2 sqrt 10)/60).
//
// Population order (an interface: kernels, host code and every caller index
// populations this way): rows in printed order; a row with several sign
// choices expands to all sign patterns of its non-zero components in
// lexicographic order, + before -, first component outermost; a "(cyc)" row
// expands to the printed vector, then (c, a, b), then (b, c, a); product sets
// enumerate the 1D nodes (0, +a, -a[, +b, -b]) with the first axis outermost.
//
// Each table stores xh = xi / c_s (dimensionless), which does not change when
// the set is rescaled to another speed of sound, plus the table's own c_s.
#pragma once

#include <cstdint>

namespace lbm {

enum SetId : int { D2Q9 = 0, D2Q19, D2Q25, D3Q13, D3Q21, D3Q27, D3V27, D3Q45, NUM_SETS };

constexpr int MAXQ = 45;

struct SetTable {
  int D, Q, degree;
  double cs;             // the table's speed of sound
  double w[MAXQ];
  double xh[MAXQ][3];    // xi / c_s
};

namespace detail {

struct Builder {
  SetTable t{};
  constexpr void add(double w, double x, double y, double z) {
    t.w[t.Q] = w;
    t.xh[t.Q][0] = x / t.cs;
    t.xh[t.Q][1] = y / t.cs;
    t.xh[t.Q][2] = z / t.cs;
    ++t.Q;
  }
  // every sign pattern of the non-zero components, + before -, first outermost
  constexpr void signs(double w, double x, double y, double z) {
    const double v[3] = {x, y, z};
    int idx[3] = {0, 0, 0};
    int k = 0;
    for (int a = 0; a < 3; ++a)
      if (v[a] != 0.0) idx[k++] = a;
    for (int pat = 0; pat < (1 << k); ++pat) {
      double o[3] = {v[0], v[1], v[2]};
      for (int b = 0; b < k; ++b)
        if ((pat >> (k - 1 - b)) & 1) o[idx[b]] = -o[idx[b]];
      add(w, o[0], o[1], o[2]);
    }
  }
  constexpr void cyclic(double w, double a, double b, double c) {
    signs(w, a, b, c);
    signs(w, c, a, b);
    signs(w, b, c, a);
  }
  constexpr void product(int D, int m, const double* node, const double* wt) {
    int total = 1;
    for (int a = 0; a < D; ++a) total *= m;
    for (int e = 0; e < total; ++e) {
      int idx[3] = {0, 0, 0};
      int r = e;
      for (int a = D - 1; a >= 0; --a) {
        idx[a] = r % m;
        r /= m;
      }
      double w = 1.0;
      double x[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < D; ++a) {
        w *= wt[idx[a]];
        x[a] = node[idx[a]];
      }
      add(w, x[0], x[1], x[2]);
    }
  }
};

// 1/sqrt(3), sqrt(3/5), golden ratio, icosahedron radii, D1Q5 roots and weights
constexpr double INV_SQRT3 = 0.5773502691896258;
constexpr double SQRT_3_5 = 0.7745966692414834;
constexpr double PHI = 1.618033988749895;
constexpr double INV_PHI = 0.6180339887498948;
constexpr double ICO_R = 1.902113032590307;   // sqrt((5 + sqrt 5) / 2)
constexpr double ICO_S = 1.1755705045849463;  // sqrt((5 - sqrt 5) / 2)
constexpr double Q5_A = 1.3556261799742657;   // sqrt(5 - sqrt 10)
constexpr double Q5_B = 2.8569700138728056;   // sqrt(5 + sqrt 10)
constexpr double Q5_WA = 0.22207592200561266; // (7 + 2 sqrt 10) / 60
constexpr double Q5_WB = 0.011257411327720682; // (7 - 2 sqrt 10) / 60

constexpr SetTable make(int id) {
  Builder b{};
  switch (id) {
  case D2Q9:
  case D3Q27: {
    const double node[3] = {0.0, 1.0, -1.0};
    const double wt[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
    b.t.D = (id == D2Q9) ? 2 : 3;
    b.t.degree = 5;
    b.t.cs = INV_SQRT3;
    b.product(b.t.D, 3, node, wt);
    break;
  }
  case D2Q25: {
    const double node[5] = {0.0, Q5_A, -Q5_A, Q5_B, -Q5_B};
    const double wt[5] = {8.0 / 15.0, Q5_WA, Q5_WA, Q5_WB, Q5_WB};
    b.t.D = 2;
    b.t.degree = 9;
    b.t.cs = 1.0;
    b.product(2, 5, node, wt);
    break;
  }
  case D2Q19:
    b.t.D = 2; b.t.degree = 9; b.t.cs = 1.0;
    b.signs(0.3168437267921905, 0.0, 0.0, 0.0);
    b.signs(0.10558878375062891, 1.4869982213169028, 0.0, 0.0);
    b.signs(0.1024247123210936, 0.775196278121181, 1.367469636752619, 0.0);
    b.signs(0.00953510698543825, 2.5175897644357486, 1.105629214668943, 0.0);
    b.signs(0.006865104210104631, 0.0, 2.9213306655318734, 0.0);
    b.signs(0.002405335328939458, 1.8663975507141328, 2.6987507639352253, 0.0);
    b.signs(0.0003939393722285871, 3.8358342053914734, 0.0, 0.0);
    break;
  case D3Q13:
    b.t.D = 3; b.t.degree = 5; b.t.cs = 1.0;
    b.signs(2.0 / 5.0, 0.0, 0.0, 0.0);
    b.signs(1.0 / 20.0, 0.0, ICO_R, ICO_S);
    b.signs(1.0 / 20.0, ICO_S, 0.0, ICO_R);
    b.signs(1.0 / 20.0, ICO_R, ICO_S, 0.0);
    break;
  case D3Q21:
    b.t.D = 3; b.t.degree = 5; b.t.cs = SQRT_3_5;
    b.signs(2.0 / 5.0, 0.0, 0.0, 0.0);
    b.signs(3.0 / 100.0, 1.0, 1.0, 1.0);
    b.signs(3.0 / 100.0, 0.0, PHI, INV_PHI);
    b.signs(3.0 / 100.0, INV_PHI, 0.0, PHI);
    b.signs(3.0 / 100.0, PHI, INV_PHI, 0.0);
    break;
  case D3V27:
    b.t.D = 3; b.t.degree = 7; b.t.cs = 1.0;
    b.signs(0.31247897198654906, 0.0, 0.0, 0.0);
    b.signs(0.06338446047675325, 1.1198362860638005, 1.1198362860638005, 1.1198362860638005);
    b.cyclic(0.029035130153906134, 2.358709038202103, 0.0, 0.0);
    b.cyclic(0.0005195469396656799, 3.142130383387586, 3.142130383387586, 0.0);
    break;
  case D3Q45: {
    b.t.D = 3; b.t.degree = 9; b.t.cs = 1.0;
    const double wa = 0.20740740740740618, wb = 0.05787037037037047, wc = 0.00462962962962958,
                 wd = 0.0004629629629629939;
    const double p = 0.06386083877343968, q = 1.2239121278243665, r = 1.5766994272507744,
                 s = 0.5069610024977665, a = 2.403092127540177, c = 0.8892242114059369,
                 d = 1.5602655313772367, e = 0.4744978678080795, f = 2.9239876105912574,
                 g = 1.7320508075688787, h = 2.7367507163016924, k = 0.14279717659756475,
                 m = 3.5256070994177073, n = 1.1335992635264445;
    b.add(wa, 0.0, 0.0, 0.0);
    b.add(wb, p, -q, -q);  b.add(wb, -p, q, q);   b.add(wb, q, -p, q);   b.add(wb, -q, p, -q);
    b.add(wb, q, q, -p);   b.add(wb, -q, -q, p);  b.add(wb, r, -s, -s);  b.add(wb, -r, s, s);
    b.add(wb, s, s, -r);   b.add(wb, -s, -s, r);  b.add(wb, -s, r, -s);  b.add(wb, s, -r, s);
    b.add(wc, a, c, -d);   b.add(wc, -a, -c, d);  b.add(wc, -a, d, -c);  b.add(wc, a, -d, c);
    b.add(wc, -c, -a, d);  b.add(wc, c, a, -d);   b.add(wc, -c, d, -a);  b.add(wc, c, -d, a);
    b.add(wc, -d, c, a);   b.add(wc, -d, a, c);   b.add(wc, d, -c, -a);  b.add(wc, d, -a, -c);
    b.add(wc, e, e, f);    b.add(wc, e, f, e);    b.add(wc, -e, -e, -f); b.add(wc, -e, -f, -e);
    b.add(wc, f, e, e);    b.add(wc, -f, -e, -e); b.add(wc, g, g, g);    b.add(wc, -g, -g, -g);
    b.add(wd, -h, k, -h);  b.add(wd, h, h, -k);   b.add(wd, h, -k, h);   b.add(wd, -h, -h, k);
    b.add(wd, k, -h, -h);  b.add(wd, -k, h, h);   b.add(wd, -m, n, n);   b.add(wd, m, -n, -n);
    b.add(wd, n, -m, n);   b.add(wd, -n, m, -n);  b.add(wd, n, n, -m);   b.add(wd, -n, -n, m);
    break;
  }
  default:
    break;
  }
  return b.t;
}

}  // namespace detail

template <int SET>
struct Set {
  static constexpr SetTable T = detail::make(SET);
  static constexpr int D = T.D;
  static constexpr int Q = T.Q;
  static constexpr int degree = T.degree;
  static constexpr double w(int i) { return T.w[i]; }
  static constexpr double xh(int i, int a) { return T.xh[i][a]; }
  static constexpr bool moves(int i, int a) { return T.xh[i][a] != 0.0; }
};

inline SetTable set_table(int id) { return detail::make(id); }

}  // namespace lbm
