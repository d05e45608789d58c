/*
 * Plain FP64 CPU oracle of the semi-Lagrangian off-lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  The GPU library never links,
 * includes or calls it, and it shares no code, header or table with the GPU
 * library: it builds its velocity sets from the printed tables of the paper,
 * takes every step in the paper's order and notation, and favours being easy
 * to check against the paper over speed.
 *
 * Paper: Wilde, Kraemer, Bedrunka, Reith, Foysi, "Cubature rules for weakly and
 * fully compressible off-lattice Boltzmann methods" (arXiv 2101.03982).
 *
 * What it computes, and where the paper defines it:
 *   - velocity sets (abscissae, weights, c_s, degree): Sec. 2, Tables
 *     tab:sets, tab:d3q13, tab:d3q21, App. C (D2Q19), App. D (D3V27), App. E
 *     (D3Q45); the Gauss-Hermite product sets D2Q9, D3Q27 (from D1Q3) and
 *     D2Q25 (from the degree-nine D1Q5) named in Sec. 1 and Table tab:sets.
 *   - semi-Lagrangian streaming: each population is interpolated at the
 *     departure point x - xi_i dt (Sec. 3, eq. sl_streaming).  The support is a
 *     uniform grid and the interpolant a tensor product of 1D Lagrange
 *     polynomials through n neighbouring nodes per axis; the sum runs over the
 *     full n^D tensor of nodes.
 *   - density and momentum (Sec. 3, eqs. density, momentum); temperature of
 *     the compressible model (Sec. 3, the energy equation with the peculiar
 *     velocity zeta = xi - u).
 *   - Hermite equilibrium as the literal tensor contraction of App. A with
 *     T0 = c_s^2 (Sec. 3, eq. for f^{eq,N}); g^eq = theta (2 C_v - D) f^eq.
 *   - BGK relaxation (Sec. 3, lattice Boltzmann equation), with
 *     tau(x) = 1/2 + (tau_ref - 1/2)/(rho theta) in the compressible model
 *     (Sec. 3: tau = mu / (c_s^2 dt P) + 1/2 with P = rho theta).
 *   - adjoint pieces for gradient checks (not in the paper): the per-cell
 *     collision Jacobian by complex-step differentiation, the transpose of
 *     streaming as an explicit scatter, and the gradient of the mean kinetic
 *     energy with respect to the initial velocity by reverse accumulation over
 *     stored states.
 *
 * Layout of every population array: [A*Q][nz][ny][nx], x fastest, A = 1
 * (f only) or 2 (f then g).  Velocity fields: [D][nz][ny][nx].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXQ 45

enum { ORC_D2Q9 = 0, ORC_D2Q19, ORC_D2Q25, ORC_D3Q13, ORC_D3Q21, ORC_D3Q27, ORC_D3V27, ORC_D3Q45, ORC_NSETS };
enum { ORC_PERIODIC = 0, ORC_EXTRAPOLATE = 1 };
/* Streaming support: a uniform grid with an n-node Lagrange stencil around
 * the departure point, or the paper's own cell-wise form: cells of p + 1
 * Gauss-Lobatto-Chebyshev support points (p = stencil - 1), neighbouring cells
 * sharing their end points. */
enum { ORC_UNIFORM = 0, ORC_GLC = 1 };

/* Configuration handed in from Python (ctypes mirror in oracle/oracle.py). */
typedef struct {
  int32_t set;          /* ORC_* set id */
  int32_t order;        /* Hermite truncation order N (2, 3, 4) */
  int32_t stencil;      /* Lagrange points per axis n (>= 1) */
  int32_t compressible; /* 0: f only, theta = 1; 1: f and g */
  int64_t nx, ny, nz;   /* grid (nz = 1 in 2D) */
  int32_t bc[3];        /* per axis: ORC_PERIODIC or ORC_EXTRAPOLATE */
  int32_t kind;         /* ORC_UNIFORM or ORC_GLC (streaming support, below) */
  double dx, dt;        /* grid spacing and time step */
  double cs;            /* target speed of sound (<= 0: the table's own) */
  double tau;           /* relaxation time (at rho theta = 1 when compressible) */
  double gamma;         /* heat capacity ratio (compressible) */
  double prandtl;       /* Prandtl number of the compressible model (<= 0 or 1: plain BGK) */
} orc_cfg;

typedef struct {
  int D, Q, degree;
  double cs_tab;
  double w[ORC_MAXQ];
  double xi[ORC_MAXQ][3];
} orc_table;

/* ------------------------------------------------------------------------ */
/* Velocity sets                                                            */
/* ------------------------------------------------------------------------ */

/* Append every sign pattern of the non-zero components of v, in
 * lexicographic order with + before - (first component outermost). */
static void push_signs(orc_table *t, double w, const double v[3], int D) {
  int nz_idx[3], k = 0;
  for (int a = 0; a < D; ++a)
    if (v[a] != 0.0) nz_idx[k++] = a;
  for (int pat = 0; pat < (1 << k); ++pat) {
    double x[3] = {v[0], v[1], v[2]};
    for (int b = 0; b < k; ++b) {
      /* bit (k-1-b) of pat: 0 -> +, 1 -> -, first component most significant */
      if ((pat >> (k - 1 - b)) & 1) x[nz_idx[b]] = -x[nz_idx[b]];
    }
    t->w[t->Q] = w;
    for (int a = 0; a < 3; ++a) t->xi[t->Q][a] = (a < D) ? x[a] : 0.0;
    t->Q++;
  }
}

/* A row printed with "(cyc)": the printed vector, then its cyclic shifts
 * (a, b, c) -> (c, a, b) -> (b, c, a), the order Tables tab:d3q13 and
 * tab:d3q21 spell out explicitly. */
static void push_cyclic(orc_table *t, double w, const double v[3]) {
  double c0[3] = {v[0], v[1], v[2]};
  double c1[3] = {v[2], v[0], v[1]};
  double c2[3] = {v[1], v[2], v[0]};
  push_signs(t, w, c0, 3);
  push_signs(t, w, c1, 3);
  push_signs(t, w, c2, 3);
}

/* Gauss-Hermite product rule of a 1D rule (Sec. 1: D1Q3 -> D2Q9 -> D3Q27). */
static void push_product(orc_table *t, int D, int m, const double *node, const double *wt) {
  int idx[3] = {0, 0, 0};
  int total = 1;
  for (int a = 0; a < D; ++a) total *= m;
  for (int e = 0; e < total; ++e) {
    int r = e;
    for (int a = D - 1; a >= 0; --a) { idx[a] = r % m; r /= m; }
    double w = 1.0;
    for (int a = 0; a < D; ++a) w *= wt[idx[a]];
    t->w[t->Q] = w;
    for (int a = 0; a < 3; ++a) t->xi[t->Q][a] = (a < D) ? node[idx[a]] : 0.0;
    t->Q++;
  }
}

static int build_table(int set, orc_table *t) {
  memset(t, 0, sizeof(*t));
  switch (set) {
  case ORC_D2Q9:
  case ORC_D3Q27: {
    /* D1Q3: roots of He_3 (0, +-sqrt 3) with weights 2/3, 1/6 at c_s = 1; in
     * lattice units the nodes are 0, +-1 and c_s = 1/sqrt 3. */
    const double node[3] = {0.0, 1.0, -1.0};
    const double wt[3] = {2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0};
    t->D = (set == ORC_D2Q9) ? 2 : 3;
    t->degree = 5;
    t->cs_tab = 1.0 / sqrt(3.0);
    push_product(t, t->D, 3, node, wt);
    return 0;
  }
  case ORC_D2Q25: {
    /* Degree-nine D1Q5: roots of He_5 = x^5 - 10 x^3 + 15 x, i.e. 0 and
     * +-sqrt(5 -+ sqrt 10), with weights 5!/(25 He_4(x)^2). */
    const double a = sqrt(5.0 - sqrt(10.0)), b = sqrt(5.0 + sqrt(10.0));
    const double node[5] = {0.0, a, -a, b, -b};
    double wt[5];
    for (int k = 0; k < 5; ++k) {
      double x = node[k];
      double he4 = x * x * x * x - 6.0 * x * x + 3.0;
      wt[k] = 120.0 / (25.0 * he4 * he4);
    }
    t->D = 2;
    t->degree = 9;
    t->cs_tab = 1.0;
    push_product(t, 2, 5, node, wt);
    return 0;
  }
  case ORC_D2Q19: {
    /* App. C, printed digits (Haegemans-Piessens E_{2,9}^{19}). */
    t->D = 2; t->degree = 9; t->cs_tab = 1.0;
    const double r0[3] = {0.0, 0.0, 0.0};
    const double r1[3] = {1.4869982213169028, 0.0, 0.0};
    const double r2[3] = {0.775196278121181, 1.367469636752619, 0.0};
    const double r3[3] = {2.5175897644357486, 1.105629214668943, 0.0};
    const double r4[3] = {0.0, 2.9213306655318734, 0.0};
    const double r5[3] = {1.8663975507141328, 2.6987507639352253, 0.0};
    const double r6[3] = {3.8358342053914734, 0.0, 0.0};
    push_signs(t, 0.3168437267921905, r0, 2);
    push_signs(t, 0.10558878375062891, r1, 2);
    push_signs(t, 0.1024247123210936, r2, 2);
    push_signs(t, 0.00953510698543825, r3, 2);
    push_signs(t, 0.006865104210104631, r4, 2);
    push_signs(t, 0.002405335328939458, r5, 2);
    push_signs(t, 0.0003939393722285871, r6, 2);
    return 0;
  }
  case ORC_D3Q13: {
    /* Table tab:d3q13: icosahedron, r^2 = (5 + sqrt 5)/2, s^2 = (5 - sqrt 5)/2. */
    t->D = 3; t->degree = 5; t->cs_tab = 1.0;
    const double r = sqrt((5.0 + sqrt(5.0)) / 2.0), s = sqrt((5.0 - sqrt(5.0)) / 2.0);
    const double z[3] = {0.0, 0.0, 0.0};
    const double a[3] = {0.0, r, s}, b[3] = {s, 0.0, r}, c[3] = {r, s, 0.0};
    push_signs(t, 2.0 / 5.0, z, 3);
    push_signs(t, 1.0 / 20.0, a, 3);
    push_signs(t, 1.0 / 20.0, b, 3);
    push_signs(t, 1.0 / 20.0, c, 3);
    return 0;
  }
  case ORC_D3Q21: {
    /* Table tab:d3q21: dodecahedron, phi = (1 + sqrt 5)/2, c_s = sqrt(3/5). */
    t->D = 3; t->degree = 5; t->cs_tab = sqrt(3.0 / 5.0);
    const double phi = (1.0 + sqrt(5.0)) / 2.0;
    const double z[3] = {0.0, 0.0, 0.0}, one[3] = {1.0, 1.0, 1.0};
    const double a[3] = {0.0, phi, 1.0 / phi}, b[3] = {1.0 / phi, 0.0, phi}, c[3] = {phi, 1.0 / phi, 0.0};
    push_signs(t, 2.0 / 5.0, z, 3);
    push_signs(t, 3.0 / 100.0, one, 3);
    push_signs(t, 3.0 / 100.0, a, 3);
    push_signs(t, 3.0 / 100.0, b, 3);
    push_signs(t, 3.0 / 100.0, c, 3);
    return 0;
  }
  case ORC_D3V27: {
    /* App. D, printed digits (Stroud-Secrest E_{3,7}^{27}); "(cyc)" rows are
     * expanded over cyclic shifts. */
    t->D = 3; t->degree = 7; t->cs_tab = 1.0;
    const double z[3] = {0.0, 0.0, 0.0};
    const double c8[3] = {1.1198362860638005, 1.1198362860638005, 1.1198362860638005};
    const double ax[3] = {2.358709038202103, 0.0, 0.0};
    const double ed[3] = {3.142130383387586, 3.142130383387586, 0.0};
    push_signs(t, 0.31247897198654906, z, 3);
    push_signs(t, 0.06338446047675325, c8, 3);
    push_cyclic(t, 0.029035130153906134, ax);
    push_cyclic(t, 0.0005195469396656799, ed);
    return 0;
  }
  case ORC_D3Q45: {
    /* App. E, the 45 printed rows verbatim (Konyaev E_{3,9}^{45}). */
    static const double rows[45][4] = {
      {0.20740740740740618, 0.0, 0.0, 0.0},
      {0.05787037037037047, 0.06386083877343968, -1.2239121278243665, -1.2239121278243665},
      {0.05787037037037047, -0.06386083877343968, 1.2239121278243665, 1.2239121278243665},
      {0.05787037037037047, 1.2239121278243665, -0.06386083877343968, 1.2239121278243665},
      {0.05787037037037047, -1.2239121278243665, 0.06386083877343968, -1.2239121278243665},
      {0.05787037037037047, 1.2239121278243665, 1.2239121278243665, -0.06386083877343968},
      {0.05787037037037047, -1.2239121278243665, -1.2239121278243665, 0.06386083877343968},
      {0.05787037037037047, 1.5766994272507744, -0.5069610024977665, -0.5069610024977665},
      {0.05787037037037047, -1.5766994272507744, 0.5069610024977665, 0.5069610024977665},
      {0.05787037037037047, 0.5069610024977665, 0.5069610024977665, -1.5766994272507744},
      {0.05787037037037047, -0.5069610024977665, -0.5069610024977665, 1.5766994272507744},
      {0.05787037037037047, -0.5069610024977665, 1.5766994272507744, -0.5069610024977665},
      {0.05787037037037047, 0.5069610024977665, -1.5766994272507744, 0.5069610024977665},
      {0.00462962962962958, 2.403092127540177, 0.8892242114059369, -1.5602655313772367},
      {0.00462962962962958, -2.403092127540177, -0.8892242114059369, 1.5602655313772367},
      {0.00462962962962958, -2.403092127540177, 1.5602655313772367, -0.8892242114059369},
      {0.00462962962962958, 2.403092127540177, -1.5602655313772367, 0.8892242114059369},
      {0.00462962962962958, -0.8892242114059369, -2.403092127540177, 1.5602655313772367},
      {0.00462962962962958, 0.8892242114059369, 2.403092127540177, -1.5602655313772367},
      {0.00462962962962958, -0.8892242114059369, 1.5602655313772367, -2.403092127540177},
      {0.00462962962962958, 0.8892242114059369, -1.5602655313772367, 2.403092127540177},
      {0.00462962962962958, -1.5602655313772367, 0.8892242114059369, 2.403092127540177},
      {0.00462962962962958, -1.5602655313772367, 2.403092127540177, 0.8892242114059369},
      {0.00462962962962958, 1.5602655313772367, -0.8892242114059369, -2.403092127540177},
      {0.00462962962962958, 1.5602655313772367, -2.403092127540177, -0.8892242114059369},
      {0.00462962962962958, 0.4744978678080795, 0.4744978678080795, 2.9239876105912574},
      {0.00462962962962958, 0.4744978678080795, 2.9239876105912574, 0.4744978678080795},
      {0.00462962962962958, -0.4744978678080795, -0.4744978678080795, -2.9239876105912574},
      {0.00462962962962958, -0.4744978678080795, -2.9239876105912574, -0.4744978678080795},
      {0.00462962962962958, 2.9239876105912574, 0.4744978678080795, 0.4744978678080795},
      {0.00462962962962958, -2.9239876105912574, -0.4744978678080795, -0.4744978678080795},
      {0.00462962962962958, 1.7320508075688787, 1.7320508075688787, 1.7320508075688787},
      {0.00462962962962958, -1.7320508075688787, -1.7320508075688787, -1.7320508075688787},
      {0.0004629629629629939, -2.7367507163016924, 0.14279717659756475, -2.7367507163016924},
      {0.0004629629629629939, 2.7367507163016924, 2.7367507163016924, -0.14279717659756475},
      {0.0004629629629629939, 2.7367507163016924, -0.14279717659756475, 2.7367507163016924},
      {0.0004629629629629939, -2.7367507163016924, -2.7367507163016924, 0.14279717659756475},
      {0.0004629629629629939, 0.14279717659756475, -2.7367507163016924, -2.7367507163016924},
      {0.0004629629629629939, -0.14279717659756475, 2.7367507163016924, 2.7367507163016924},
      {0.0004629629629629939, -3.5256070994177073, 1.1335992635264445, 1.1335992635264445},
      {0.0004629629629629939, 3.5256070994177073, -1.1335992635264445, -1.1335992635264445},
      {0.0004629629629629939, 1.1335992635264445, -3.5256070994177073, 1.1335992635264445},
      {0.0004629629629629939, -1.1335992635264445, 3.5256070994177073, -1.1335992635264445},
      {0.0004629629629629939, 1.1335992635264445, 1.1335992635264445, -3.5256070994177073},
      {0.0004629629629629939, -1.1335992635264445, -1.1335992635264445, 3.5256070994177073},
    };
    t->D = 3; t->degree = 9; t->cs_tab = 1.0; t->Q = 45;
    for (int i = 0; i < 45; ++i) {
      t->w[i] = rows[i][0];
      for (int a = 0; a < 3; ++a) t->xi[i][a] = rows[i][1 + a];
    }
    return 0;
  }
  default:
    return -1;
  }
}

/* Exported: the table as the oracle builds it (unscaled, table units). */
int orc_set_table(int set, int32_t *Q, int32_t *D, int32_t *degree, double *cs_tab, double *w, double *xi) {
  orc_table t;
  if (build_table(set, &t)) return -1;
  *Q = t.Q; *D = t.D; *degree = t.degree; *cs_tab = t.cs_tab;
  for (int i = 0; i < t.Q; ++i) {
    w[i] = t.w[i];
    for (int a = 0; a < 3; ++a) xi[3 * i + a] = t.xi[i][a];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Problem setup                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_cfg c;
  orc_table t;       /* xi scaled to the target c_s */
  int D, Q, A;
  double cs, T0, Cv;
  int64_t n[3], ncell;
} orc_prob;

static int setup(const orc_cfg *c, orc_prob *p) {
  memset(p, 0, sizeof(*p));
  p->c = *c;
  if (build_table(c->set, &p->t)) return -1;
  p->D = p->t.D;
  p->Q = p->t.Q;
  p->A = c->compressible ? 2 : 1;
  /* Sec. 2: velocity sets are rescaled to the wanted speed of sound. */
  p->cs = (c->cs > 0.0) ? c->cs : p->t.cs_tab;
  double lam = p->cs / p->t.cs_tab;
  for (int i = 0; i < p->Q; ++i)
    for (int a = 0; a < 3; ++a) p->t.xi[i][a] *= lam;
  p->T0 = p->cs * p->cs; /* reference temperature, T0 = c_s^2 */
  p->Cv = c->compressible ? 1.0 / (c->gamma - 1.0) : 0.5 * p->D;
  p->n[0] = c->nx; p->n[1] = c->ny; p->n[2] = (p->D == 3) ? c->nz : 1;
  p->ncell = p->n[0] * p->n[1] * p->n[2];
  if (c->order < 0 || c->order > 4 || c->stencil < 1) return -1;
  if (c->kind == ORC_GLC) {
    /* every axis is a whole number of periodic cells of p nodes */
    const int pp = c->stencil - 1;
    if (pp < 1 || pp > 7) return -1;
    for (int a = 0; a < p->D; ++a)
      if (p->n[a] % pp != 0 || c->bc[a] != ORC_PERIODIC) return -1;
  } else if (c->kind != ORC_UNIFORM) {
    return -1;
  }
  return 0;
}

static inline int64_t cell_index(const orc_prob *p, const int64_t x[3]) {
  return (x[2] * p->n[1] + x[1]) * p->n[0] + x[0];
}

static inline void cell_coords(const orc_prob *p, int64_t e, int64_t x[3]) {
  x[0] = e % p->n[0];
  x[1] = (e / p->n[0]) % p->n[1];
  x[2] = e / (p->n[0] * p->n[1]);
}

/* Map an unwrapped node index onto the grid: periodic wrap, or zeroth-order
 * extrapolation (the nearest boundary node) on an open axis. */
static inline int64_t wrap_node(const orc_prob *p, int axis, int64_t m) {
  int64_t N = p->n[axis];
  if (p->c.bc[axis] == ORC_EXTRAPOLATE) {
    if (m < 0) return 0;
    if (m >= N) return N - 1;
    return m;
  }
  int64_t r = m % N;
  return (r < 0) ? r + N : r;
}

/* The n 1D Lagrange nodes around the departure coordinate d = j - s of arrival
 * node j (s = shift in cells), and their weights
 *   L_k(d) = prod_{m != k} (d - x_m) / (x_k - x_m).
 * Even n: the n/2 nodes on either side of d.  Odd n: centred on the node
 * nearest to d; when d lies exactly half-way, the node on the arrival side.
 * The differences d - x_m are formed as (j - x_m) - s, exact integers minus s,
 * so that the weights do not depend on the magnitude of j. */
static void stencil_1d(int64_t j, double s, int n, int64_t *nodes, double *L) {
  int64_t first;
  double r = -s;                 /* d - j */
  if (n % 2 == 0) {
    int64_t fl = (int64_t)floor(r);  /* floor(d) - j */
    first = j + fl - n / 2 + 1;
  } else {
    int64_t fl = (int64_t)floor(r);
    double frac = r - (double)fl;
    int64_t c;
    if (frac < 0.5) c = fl;
    else if (frac > 0.5) c = fl + 1;
    else c = (llabs(fl) <= llabs(fl + 1)) ? fl : fl + 1; /* tie: nearer to j */
    first = j + c - (n - 1) / 2;
  }
  for (int k = 0; k < n; ++k) nodes[k] = first + k;
  for (int k = 0; k < n; ++k) {
    double num = 1.0, den = 1.0;
    for (int m = 0; m < n; ++m) {
      if (m == k) continue;
      num *= (double)(j - nodes[m]) - s;
      den *= (double)(nodes[k] - nodes[m]);
    }
    L[k] = num / den;
  }
}

static inline double shift_of(const orc_prob *p, int i, int axis) {
  return p->t.xi[i][axis] * p->c.dt / p->c.dx;
}

/* Gauss-Lobatto-Chebyshev support point m of a cell of order pp, in cell
 * units: the extrema of the Chebyshev polynomial T_pp mapped onto [0, 1]
 * (Sec. 3: the support points of the paper's cell-wise interpolation). */
static inline double glc_point(int m, int pp) {
  const double pi = 3.14159265358979323846;
  return 0.5 * (1.0 - cos(pi * (double)m / (double)pp));
}

/* Cell-wise streaming (Sec. 3, eq. sl_streaming): node j is support point k
 * of cell c (j = c pp + k; the cell's last point is the next cell's first).
 * Its departure point lies s nodes' mean spacing upstream, i.e. s / pp cells,
 * at r = glc_point(k) - s / pp cells from the start of cell c.  The cell that
 * holds it is c + floor(r); the value there is the interpolation polynomial
 * of that cell, sum_t psi_t(eta) f(node t of the cell), with eta the
 * departure point's coordinate in the cell and psi_t the Lagrange
 * polynomials through the cell's pp + 1 support points. */
static void stencil_glc(int64_t j, double s, int pp, int64_t *nodes, double *L) {
  int64_t c = j / pp, k = j % pp;
  if (k < 0) { k += pp; c -= 1; }
  const double r = glc_point((int)k, pp) - s / (double)pp;
  const double d = floor(r);
  const double eta = r - d;
  const int64_t first = (c + (int64_t)d) * pp;
  for (int t = 0; t <= pp; ++t) nodes[t] = first + t;
  for (int t = 0; t <= pp; ++t) {
    double num = 1.0, den = 1.0;
    for (int m = 0; m <= pp; ++m) {
      if (m == t) continue;
      num *= eta - glc_point(m, pp);
      den *= glc_point(t, pp) - glc_point(m, pp);
    }
    L[t] = num / den;
  }
}

/* The nodes and weights of population i's interpolation along `axis` for
 * arrival node j, for either streaming support; returns the node count. */
static int axis_stencil(const orc_prob *p, int i, int axis, int64_t j, int64_t *nodes, double *L) {
  const int n = p->c.stencil;
  if (p->c.kind == ORC_GLC) {
    stencil_glc(j, shift_of(p, i, axis), n - 1, nodes, L);
    return n;
  }
  stencil_1d(j, shift_of(p, i, axis), n, nodes, L);
  return n;
}

/* ------------------------------------------------------------------------ */
/* Streaming (Sec. 3, eq. sl_streaming): full tensor-product sum             */
/* ------------------------------------------------------------------------ */

static double interp_at(const orc_prob *p, const double *fi, int i, const int64_t x[3]) {
  int64_t nodes[3][8];
  double L[3][8];
  int na[3] = {1, 1, 1};
  for (int a = 0; a < 3; ++a) {
    if (a < p->D) {
      na[a] = axis_stencil(p, i, a, x[a], nodes[a], L[a]);
    } else {
      nodes[a][0] = 0;
      L[a][0] = 1.0;
    }
  }
  double sum = 0.0;
  for (int kz = 0; kz < na[2]; ++kz)
    for (int ky = 0; ky < na[1]; ++ky)
      for (int kx = 0; kx < na[0]; ++kx) {
        int64_t m[3] = {wrap_node(p, 0, nodes[0][kx]), wrap_node(p, 1, nodes[1][ky]),
                        (p->D == 3) ? wrap_node(p, 2, nodes[2][kz]) : 0};
        sum += L[0][kx] * L[1][ky] * L[2][kz] * fi[cell_index(p, m)];
      }
  return sum;
}

int orc_stream(const orc_cfg *c, const double *f, double *ft) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  for (int a = 0; a < p.A; ++a)
    for (int i = 0; i < p.Q; ++i) {
      const double *fi = f + (int64_t)(a * p.Q + i) * NC;
      double *oi = ft + (int64_t)(a * p.Q + i) * NC;
#pragma omp parallel for schedule(static)
      for (int64_t e = 0; e < NC; ++e) {
        int64_t x[3];
        cell_coords(&p, e, x);
        oi[e] = interp_at(&p, fi, i, x);
      }
    }
  return 0;
}

/* Transpose of streaming, as an explicit scatter: every arrival cell hands
 * mu * L back to each node of its stencil. */
int orc_stream_transpose(const orc_cfg *c, const double *mu, double *lam) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  memset(lam, 0, sizeof(double) * (size_t)(p.A * p.Q) * (size_t)NC);
  for (int a = 0; a < p.A; ++a)
    for (int i = 0; i < p.Q; ++i) {
      const double *mi = mu + (int64_t)(a * p.Q + i) * NC;
      double *li = lam + (int64_t)(a * p.Q + i) * NC;
      for (int64_t e = 0; e < NC; ++e) {
        int64_t x[3];
        cell_coords(&p, e, x);
        int64_t nodes[3][8];
        double L[3][8];
        int na[3] = {1, 1, 1};
        for (int ax = 0; ax < 3; ++ax) {
          if (ax < p.D) {
            na[ax] = axis_stencil(&p, i, ax, x[ax], nodes[ax], L[ax]);
          } else {
            nodes[ax][0] = 0;
            L[ax][0] = 1.0;
          }
        }
        for (int kz = 0; kz < na[2]; ++kz)
          for (int ky = 0; ky < na[1]; ++ky)
            for (int kx = 0; kx < na[0]; ++kx) {
              int64_t m[3] = {wrap_node(&p, 0, nodes[0][kx]), wrap_node(&p, 1, nodes[1][ky]),
                              (p.D == 3) ? wrap_node(&p, 2, nodes[2][kz]) : 0};
              li[cell_index(&p, m)] += L[0][kx] * L[1][ky] * L[2][kz] * mi[e];
            }
      }
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium: literal App. A tensors                                       */
/* ------------------------------------------------------------------------ */

static inline double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* f^{eq,N}_i = w_i sum_{n<=N} (1/n!) a^(n)_eq : H_i^(n), with
 *   H^(0) = 1, H^(1) = xh/c_s, H^(2) = (xh xh - delta)/c_s^2,
 *   H^(3) = (xh xh xh - (xh delta)_3)/c_s^3,
 *   H^(4) = (xh xh xh xh - T + Delta)/c_s^4,   xh = xi / c_s,
 *   a^(0) = rho, a^(1) = rho u, a^(2) = rho (u u + T0 eta delta),
 *   a^(3) = rho [u u u + T0 eta (delta u)_3],
 *   a^(4) = rho [u u u u + T0 eta (delta u u)_6 + T0^2 eta^2 Delta],
 * eta = theta - 1 (App. A; the fourth-order moment is read as the sum of
 * those three groups of terms).  Complex arguments carry the complex-step
 * perturbation used for derivatives; the real part is the equilibrium. */
static void feq_tensor(const orc_prob *p, double complex rho, const double complex u[3],
                       double complex theta, double complex *feq) {
  const int D = p->D, N = p->c.order;
  const double cs = p->cs, T0 = p->T0;
  const double complex eta = theta - 1.0;
  for (int i = 0; i < p->Q; ++i) {
    double xh[3];
    for (int a = 0; a < 3; ++a) xh[a] = p->t.xi[i][a] / cs;
    double complex sum = rho; /* n = 0 */
    if (N >= 1) {
      double complex s1 = 0.0;
      for (int a = 0; a < D; ++a) s1 += rho * u[a] * (xh[a] / cs);
      sum += s1;
    }
    if (N >= 2) {
      double complex s2 = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
          double complex A2 = rho * (u[a] * u[b] + T0 * eta * kd(a, b));
          double H2 = (xh[a] * xh[b] - kd(a, b)) / (cs * cs);
          s2 += A2 * H2;
        }
      sum += s2 / 2.0;
    }
    if (N >= 3) {
      double complex s3 = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
          for (int g = 0; g < D; ++g) {
            double complex A3 = rho * (u[a] * u[b] * u[g] +
                                       T0 * eta * (kd(a, b) * u[g] + kd(a, g) * u[b] + kd(b, g) * u[a]));
            double H3 = (xh[a] * xh[b] * xh[g] - (xh[a] * kd(b, g) + xh[b] * kd(a, g) + xh[g] * kd(a, b))) /
                        (cs * cs * cs);
            s3 += A3 * H3;
          }
      sum += s3 / 6.0;
    }
    if (N >= 4) {
      double complex s4 = 0.0;
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
          for (int g = 0; g < D; ++g)
            for (int d = 0; d < D; ++d) {
              double Dl = kd(a, b) * kd(g, d) + kd(a, g) * kd(b, d) + kd(a, d) * kd(b, g);
              double complex A4 =
                  rho * (u[a] * u[b] * u[g] * u[d] +
                         T0 * eta *
                             (kd(a, b) * u[g] * u[d] + kd(a, g) * u[b] * u[d] + kd(a, d) * u[b] * u[g] +
                              kd(b, g) * u[a] * u[d] + kd(b, d) * u[a] * u[g] + kd(g, d) * u[a] * u[b]) +
                         T0 * T0 * eta * eta * Dl);
              double T = xh[a] * xh[b] * kd(g, d) + xh[a] * xh[g] * kd(b, d) + xh[a] * xh[d] * kd(b, g) +
                         xh[b] * xh[g] * kd(a, d) + xh[b] * xh[d] * kd(a, g) + xh[g] * xh[d] * kd(a, b);
              double H4 = (xh[a] * xh[b] * xh[g] * xh[d] - T + Dl) / (cs * cs * cs * cs);
              s4 += A4 * H4;
            }
      sum += s4 / 24.0;
    }
    feq[i] = p->t.w[i] * sum;
  }
}

/* Equilibria of f (and g) for given macroscopic values; g^eq = theta (2 C_v - D) f^eq. */
static void equilibria(const orc_prob *p, double complex rho, const double complex u[3],
                       double complex theta, double complex *out) {
  feq_tensor(p, rho, u, theta, out);
  if (p->A == 2)
    for (int i = 0; i < p->Q; ++i) out[p->Q + i] = theta * (2.0 * p->Cv - p->D) * out[i];
}

/* Density, velocity and temperature of one cell's populations
 * (Sec. 3: rho = sum f, rho u = sum xi f,
 *  2 rho C_v theta = sum (|xi - u|^2 f / T0 + g)). */
static void macroscopic(const orc_prob *p, const double complex *fc, double complex *rho,
                        double complex u[3], double complex *theta) {
  double complex r = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < p->Q; ++i) {
    r += fc[i];
    for (int a = 0; a < p->D; ++a) j[a] += p->t.xi[i][a] * fc[i];
  }
  for (int a = 0; a < 3; ++a) u[a] = (a < p->D) ? j[a] / r : 0.0;
  *rho = r;
  if (p->A == 2) {
    double complex e = 0.0;
    for (int i = 0; i < p->Q; ++i) {
      double complex z2 = 0.0;
      for (int a = 0; a < p->D; ++a) {
        double complex z = p->t.xi[i][a] - u[a];
        z2 += z * z;
      }
      e += z2 * fc[i] / p->T0 + fc[p->Q + i];
    }
    *theta = e / (2.0 * r * p->Cv);
  } else {
    *theta = 1.0;
  }
}

/* Quasi-equilibrium of the compressible model for a Prandtl number other than
 * one (Sec. 3 names a quasi-equilibrium approach for varying Pr without
 * describing it; this is the reading stated with the repository's design
 * notes).  The heat is carried by the contracted third moment of f and the
 * first moment of g; their non-equilibrium parts in the frame moving with the
 * fluid are
 *   q_f = sum_i zeta_i |zeta_i|^2 (f_i - f^eq_i),  q_g = sum_i zeta_i (g_i - g^eq_i),
 * zeta_i = xi_i - u.  The quasi-equilibrium equals the equilibrium except that
 * these fluxes take their present values:
 *   f*_i = f^eq_i + w_i (xh_i . q_f / c_s^3) (|xh_i|^2 - (D + 2)) / (2 (D + 2)),
 *   g*_i = g^eq_i + w_i (xh_i . q_g / c_s),  xh = xi / c_s;
 * the added terms are odd in xi, so they carry no mass, momentum, stress or
 * energy, and (for sets exact to degree six) exactly the fluxes q_f, q_g. */
static void quasi_equilibrium(const orc_prob *p, const double complex *fin, const double complex *eq,
                              const double complex u[3], double complex *qe) {
  const int D = p->D, Q = p->Q;
  const double cs = p->cs;
  double complex qf[3] = {0.0, 0.0, 0.0}, qg[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < Q; ++i) {
    double complex zeta[3], z2 = 0.0;
    for (int a = 0; a < D; ++a) {
      zeta[a] = p->t.xi[i][a] - u[a];
      z2 += zeta[a] * zeta[a];
    }
    for (int a = 0; a < D; ++a) {
      qf[a] += zeta[a] * z2 * (fin[i] - eq[i]);
      qg[a] += zeta[a] * (fin[Q + i] - eq[Q + i]);
    }
  }
  for (int i = 0; i < Q; ++i) {
    double xh[3], X = 0.0;
    for (int a = 0; a < D; ++a) {
      xh[a] = p->t.xi[i][a] / cs;
      X += xh[a] * xh[a];
    }
    double complex pf = 0.0, pg = 0.0;
    for (int a = 0; a < D; ++a) {
      pf += xh[a] * qf[a] / (cs * cs * cs);
      pg += xh[a] * qg[a] / cs;
    }
    qe[i] = eq[i] + p->t.w[i] * pf * (X - (D + 2.0)) / (2.0 * (D + 2.0));
    qe[Q + i] = eq[Q + i] + p->t.w[i] * pg;
  }
}

/* BGK collision of one cell (Sec. 3): f* = f - (f - f^eq)/tau.  Compressible
 * model with Pr != 1: f* = f - (f - f^eq)/tau + (1/tau - 1/tau_q)(f^qe - f^eq)
 * (and the same for g), tau_q = 1/2 + (tau - 1/2)/Pr, so that the heat fluxes
 * q_f, q_g relax at 1/tau_q and every other moment at 1/tau. */
static void collide_cell(const orc_prob *p, const double complex *fin, double complex *fout) {
  double complex rho, u[3], theta, eq[2 * ORC_MAXQ];
  macroscopic(p, fin, &rho, u, &theta);
  equilibria(p, rho, u, theta, eq);
  double complex tau = p->c.tau;
  if (p->A == 2) tau = 0.5 + (p->c.tau - 0.5) / (rho * theta); /* P = rho theta */
  for (int k = 0; k < p->A * p->Q; ++k) fout[k] = fin[k] - (fin[k] - eq[k]) / tau;
  if (p->A == 2 && p->c.prandtl > 0.0 && p->c.prandtl != 1.0) {
    double complex qe[2 * ORC_MAXQ];
    quasi_equilibrium(p, fin, eq, u, qe);
    const double complex tau_q = 0.5 + (tau - 0.5) / p->c.prandtl;
    for (int k = 0; k < 2 * p->Q; ++k) fout[k] += (1.0 / tau - 1.0 / tau_q) * (qe[k] - eq[k]);
  }
}

int orc_collide(const orc_cfg *c, const double *ft, double *fc) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < NC; ++e) {
    double complex in[2 * ORC_MAXQ], out[2 * ORC_MAXQ];
    for (int k = 0; k < AQ; ++k) in[k] = ft[(int64_t)k * NC + e];
    collide_cell(&p, in, out);
    for (int k = 0; k < AQ; ++k) fc[(int64_t)k * NC + e] = creal(out[k]);
  }
  return 0;
}

/* One time step: stream, then collide.  The stored state is post-collision. */
int orc_step(const orc_cfg *c, const double *f, double *fout, double *scratch) {
  if (orc_stream(c, f, scratch)) return -1;
  return orc_collide(c, scratch, fout);
}

/* nsteps steps in place; scratch holds two more states. */
int orc_run(const orc_cfg *c, double *f, int64_t nsteps, double *scratch) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const size_t bytes = sizeof(double) * (size_t)(p.A * p.Q) * (size_t)p.ncell;
  double *tmp = scratch, *nxt = scratch + (size_t)(p.A * p.Q) * (size_t)p.ncell;
  for (int64_t s = 0; s < nsteps; ++s) {
    if (orc_step(c, f, nxt, tmp)) return -1;
    memcpy(f, nxt, bytes);
  }
  return 0;
}

/* Populations at equilibrium with the given fields (theta may be NULL: 1). */
int orc_init(const orc_cfg *c, const double *rho, const double *u, const double *theta, double *f) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < NC; ++e) {
    double complex uu[3] = {0.0, 0.0, 0.0}, eq[2 * ORC_MAXQ];
    for (int a = 0; a < p.D; ++a) uu[a] = u[(int64_t)a * NC + e];
    double complex th = theta ? theta[e] : 1.0;
    equilibria(&p, rho[e], uu, th, eq);
    for (int k = 0; k < AQ; ++k) f[(int64_t)k * NC + e] = creal(eq[k]);
  }
  return 0;
}

/* Per-cell rho, u, theta of a stored state, and global diagnostics:
 * diag[0] = sum rho, diag[1..3] = sum rho u, diag[4] = mean |u|^2 / 2,
 * diag[5] = sum of the total energy moment sum(|xi|^2 f / T0 + g) / 2,
 * diag[6] = min rho, diag[7] = min theta. */
int orc_moments(const orc_cfg *c, const double *f, double *rho, double *u, double *theta, double *diag) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
  double mass = 0.0, mom[3] = {0, 0, 0}, ke = 0.0, en = 0.0, rmin = INFINITY, tmin = INFINITY;
  for (int64_t e = 0; e < NC; ++e) {
    double complex fc[2 * ORC_MAXQ], r, uu[3], th;
    for (int k = 0; k < AQ; ++k) fc[k] = f[(int64_t)k * NC + e];
    macroscopic(&p, fc, &r, uu, &th);
    double rr = creal(r), t = creal(th), u2 = 0.0;
    if (rho) rho[e] = rr;
    for (int a = 0; a < p.D; ++a) {
      if (u) u[(int64_t)a * NC + e] = creal(uu[a]);
      mom[a] += rr * creal(uu[a]);
      u2 += creal(uu[a]) * creal(uu[a]);
    }
    if (theta) theta[e] = t;
    mass += rr;
    ke += 0.5 * u2;
    double ee = 0.0;
    for (int i = 0; i < p.Q; ++i) {
      double x2 = 0.0;
      for (int a = 0; a < p.D; ++a) x2 += p.t.xi[i][a] * p.t.xi[i][a];
      ee += x2 * creal(fc[i]) / p.T0 + ((p.A == 2) ? creal(fc[p.Q + i]) : 0.0);
    }
    en += 0.5 * ee;
    if (rr < rmin) rmin = rr;
    if (t < tmin) tmin = t;
  }
  diag[0] = mass;
  diag[1] = mom[0]; diag[2] = mom[1]; diag[3] = mom[2];
  diag[4] = ke / (double)NC;
  diag[5] = en;
  diag[6] = rmin;
  diag[7] = tmin;
  return 0;
}

/* Equilibrium of one cell, real values (for tests of App. A). */
int orc_feq(const orc_cfg *c, double rho, const double *u, double theta, double *out) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  double complex uu[3] = {0.0, 0.0, 0.0}, eq[2 * ORC_MAXQ];
  for (int a = 0; a < p.D; ++a) uu[a] = u[a];
  equilibria(&p, rho, uu, theta, eq);
  for (int k = 0; k < p.A * p.Q; ++k) out[k] = creal(eq[k]);
  return 0;
}

/* Collision of one cell, real values. */
int orc_collide_one(const orc_cfg *c, const double *in, double *out) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  double complex a[2 * ORC_MAXQ], b[2 * ORC_MAXQ];
  for (int k = 0; k < p.A * p.Q; ++k) a[k] = in[k];
  collide_cell(&p, a, b);
  for (int k = 0; k < p.A * p.Q; ++k) out[k] = creal(b[k]);
  return 0;
}

/* One step evaluated at selected cells only, starting from the equilibrium of
 * the given initial fields: the populations of every stencil node are formed
 * on the fly, so full-size grids need no full-size oracle state.
 * out: [ncells][A*Q]. */
int orc_first_step_at(const orc_cfg *c, const double *rho, const double *u, const double *theta,
                      const int64_t *cells, int64_t ncells, double *out) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
#pragma omp parallel for schedule(dynamic)
  for (int64_t s = 0; s < ncells; ++s) {
    int64_t x[3];
    cell_coords(&p, cells[s], x);
    double complex ft[2 * ORC_MAXQ], fo[2 * ORC_MAXQ];
    for (int a = 0; a < p.A; ++a)
      for (int i = 0; i < p.Q; ++i) {
        int64_t nodes[3][8];
        double L[3][8];
        int na[3] = {1, 1, 1};
        for (int ax = 0; ax < 3; ++ax) {
          if (ax < p.D) {
            na[ax] = axis_stencil(&p, i, ax, x[ax], nodes[ax], L[ax]);
          } else {
            nodes[ax][0] = 0;
            L[ax][0] = 1.0;
          }
        }
        double sum = 0.0;
        for (int kz = 0; kz < na[2]; ++kz)
          for (int ky = 0; ky < na[1]; ++ky)
            for (int kx = 0; kx < na[0]; ++kx) {
              int64_t m[3] = {wrap_node(&p, 0, nodes[0][kx]), wrap_node(&p, 1, nodes[1][ky]),
                              (p.D == 3) ? wrap_node(&p, 2, nodes[2][kz]) : 0};
              int64_t e = cell_index(&p, m);
              double complex uu[3] = {0.0, 0.0, 0.0}, eq[2 * ORC_MAXQ];
              for (int b = 0; b < p.D; ++b) uu[b] = u[(int64_t)b * NC + e];
              equilibria(&p, rho[e], uu, theta ? theta[e] : 1.0, eq);
              sum += L[0][kx] * L[1][ky] * L[2][kz] * creal(eq[a * p.Q + i]);
            }
        ft[a * p.Q + i] = sum;
      }
    collide_cell(&p, ft, fo);
    for (int k = 0; k < AQ; ++k) out[s * AQ + k] = creal(fo[k]);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Adjoint pieces (gradient checks; not part of the paper)                  */
/* ------------------------------------------------------------------------ */

#define ORC_CSTEP 1e-30

/* Dense Jacobian of one cell's collision, J[r][k] = d f*_r / d f~_k, by
 * complex-step differentiation (exact to rounding). */
static void jacobian_cell(const orc_prob *p, const double *in, double *J) {
  const int AQ = p->A * p->Q;
  for (int k = 0; k < AQ; ++k) {
    double complex a[2 * ORC_MAXQ], b[2 * ORC_MAXQ];
    for (int r = 0; r < AQ; ++r) a[r] = in[r];
    a[k] += I * ORC_CSTEP;
    collide_cell(p, a, b);
    for (int r = 0; r < AQ; ++r) J[r * AQ + k] = cimag(b[r]) / ORC_CSTEP;
  }
}

int orc_collide_jacobian(const orc_cfg *c, const double *in, double *J) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  jacobian_cell(&p, in, J);
  return 0;
}

/* nu = J_C(ft)^T lam, cell by cell, with the dense complex-step Jacobian. */
int orc_adjoint_collide(const orc_cfg *c, const double *ft, const double *lam, double *nu) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < NC; ++e) {
    double in[2 * ORC_MAXQ], J[4 * ORC_MAXQ * ORC_MAXQ];
    for (int k = 0; k < AQ; ++k) in[k] = ft[(int64_t)k * NC + e];
    jacobian_cell(&p, in, J);
    for (int k = 0; k < AQ; ++k) {
      double s = 0.0;
      for (int r = 0; r < AQ; ++r) s += J[r * AQ + k] * lam[(int64_t)r * NC + e];
      nu[(int64_t)k * NC + e] = s;
    }
  }
  return 0;
}

/* Mean kinetic energy k = <|u|^2/2> over the nodes (Sec. 4.2, without density
 * weighting) of a stored state, and its gradient with respect to every
 * population (complex step per population). */
int orc_ke_and_grad(const orc_cfg *c, const double *f, double *ke, double *grad) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
  double total = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : total)
  for (int64_t e = 0; e < NC; ++e) {
    double complex fc[2 * ORC_MAXQ], r, uu[3], th;
    for (int k = 0; k < AQ; ++k) fc[k] = f[(int64_t)k * NC + e];
    macroscopic(&p, fc, &r, uu, &th);
    double u2 = 0.0;
    for (int a = 0; a < p.D; ++a) u2 += creal(uu[a]) * creal(uu[a]);
    total += 0.5 * u2;
    if (grad) {
      for (int k = 0; k < AQ; ++k) {
        double complex g[2 * ORC_MAXQ];
        for (int m = 0; m < AQ; ++m) g[m] = fc[m];
        g[k] += I * ORC_CSTEP;
        macroscopic(&p, g, &r, uu, &th);
        double complex k2 = 0.0;
        for (int a = 0; a < p.D; ++a) k2 += uu[a] * uu[a];
        grad[(int64_t)k * NC + e] = cimag(0.5 * k2) / ORC_CSTEP / (double)NC;
      }
    }
  }
  *ke = total / (double)NC;
  return 0;
}

/* d L / d u0 from lam0 = d L / d f0 through f0 = f^eq(rho0, u0, theta0),
 * with rho0 and theta0 held fixed (complex step per velocity component). */
int orc_init_transpose(const orc_cfg *c, const double *rho, const double *u, const double *theta,
                       const double *lam0, double *grad_u) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const int64_t NC = p.ncell;
  const int AQ = p.A * p.Q;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < NC; ++e) {
    for (int b = 0; b < p.D; ++b) {
      double complex uu[3] = {0.0, 0.0, 0.0}, eq[2 * ORC_MAXQ];
      for (int a = 0; a < p.D; ++a) uu[a] = u[(int64_t)a * NC + e];
      uu[b] += I * ORC_CSTEP;
      equilibria(&p, rho[e], uu, theta ? theta[e] : 1.0, eq);
      double s = 0.0;
      for (int k = 0; k < AQ; ++k) s += cimag(eq[k]) / ORC_CSTEP * lam0[(int64_t)k * NC + e];
      grad_u[(int64_t)b * NC + e] = s;
    }
  }
  return 0;
}

/* Loss k(f_T) after nsteps steps from f0 = f^eq(rho0, u0, theta0) and its
 * gradient with respect to u0, by reverse accumulation over all stored
 * states: lam_T = dk/df_T; for each step backwards nu = J_C(S f)^T lam,
 * lam = S^T nu; finally through the initial equilibrium. */
int orc_ke_gradient_u0(const orc_cfg *c, const double *rho, const double *u, const double *theta,
                       int64_t nsteps, double *loss, double *grad_u) {
  orc_prob p;
  if (setup(c, &p)) return -1;
  const size_t S = (size_t)(p.A * p.Q) * (size_t)p.ncell;
  double *states = (double *)malloc(sizeof(double) * S * (size_t)(nsteps + 1));
  double *tmp = (double *)malloc(sizeof(double) * S);
  double *lam = (double *)malloc(sizeof(double) * S);
  double *nu = (double *)malloc(sizeof(double) * S);
  if (!states || !tmp || !lam || !nu) {
    free(states); free(tmp); free(lam); free(nu);
    return -2;
  }
  orc_init(c, rho, u, theta, states);
  for (int64_t s = 0; s < nsteps; ++s) orc_step(c, states + S * (size_t)s, states + S * (size_t)(s + 1), tmp);
  orc_ke_and_grad(c, states + S * (size_t)nsteps, loss, lam);
  for (int64_t s = nsteps; s >= 1; --s) {
    orc_stream(c, states + S * (size_t)(s - 1), tmp); /* f~ of step s */
    orc_adjoint_collide(c, tmp, lam, nu);
    orc_stream_transpose(c, nu, lam);
  }
  orc_init_transpose(c, rho, u, theta, lam, grad_u);
  free(states); free(tmp); free(lam); free(nu);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
