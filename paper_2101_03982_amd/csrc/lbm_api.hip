// C ABI of liblbm (include/lbm.h): argument checks, the per-direction
// stencil (computed on the host in FP64), device tables, launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_diag.hpp"
#include "lbm_dispatch.hpp"
#include "lbm_sets.hpp"

using namespace lbm;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

constexpr int MAXNS = 5;

// 1D stencil of a shift s (cells moved per step): the offset of the first node
// from the arrival node and the n Lagrange weights at the departure point.
// Departure coordinate relative to the arrival node: t0 = -s.  Even n: the
// n/2 nodes on either side; odd n: centred on the nearest node, the arrival
// side winning an exact tie (Sec. 3, eq. sl_streaming, on a uniform grid).
void stencil_axis(double s, int n, int* first, double* L) {
  const double t0 = -s;
  const double fl = std::floor(t0);
  int f;
  if (n % 2 == 0) {
    f = int(fl) - n / 2 + 1;
  } else {
    const double frac = t0 - fl;
    int c;
    if (frac < 0.5) c = int(fl);
    else if (frac > 0.5) c = int(fl) + 1;
    else c = (std::abs(fl) <= std::abs(fl + 1.0)) ? int(fl) : int(fl) + 1;
    f = c - (n - 1) / 2;
  }
  *first = f;
  const double t = t0 - double(f);  // departure point in units of cells from the first node
  for (int k = 0; k < n; ++k) {
    double num = 1.0, den = 1.0;
    for (int m = 0; m < n; ++m) {
      if (m == k) continue;
      num *= t - double(m);
      den *= double(k - m);
    }
    L[k] = num / den;
  }
}

// Rounds the weights onto a grid of 2^-bits and gives the largest one the
// remainder, so that they sum to exactly one in real arithmetic (a stencil
// whose weights do not sum to one adds or removes mass every step).
void quantize_unit_sum(double* L, int n, int bits) {
  if (n <= 1) return;
  const double q = std::ldexp(1.0, bits);
  int big = 0;
  for (int k = 1; k < n; ++k)
    if (std::abs(L[k]) > std::abs(L[big])) big = k;
  if (std::abs(L[big]) >= 1.0) return;  // grid values outside (-1, 1) may not be representable
  double rest = 0.0;
  for (int k = 0; k < n; ++k) {
    if (k == big) continue;
    L[k] = std::nearbyint(L[k] * q) / q;
    rest += L[k];
  }
  L[big] = 1.0 - rest;
}

}  // namespace

// Reduction scratch of lbm_moments_noalloc: a file-scope device array, so
// that the call allocates nothing.  Each device holds its own copy; its
// address on a device comes from hipGetSymbolAddress (the array's name in
// host code is not a device address).  Calls that overlap on one device
// share it and race.
constexpr size_t SCRATCH_DOUBLES = size_t(MOMENT_BLOCKS + 1) * NPART;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller has made it current).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) return fail(LBM_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return LBM_OK;
}

// Cell-wise streaming on Gauss-Lobatto-Chebyshev support points (Sec. 3, eq.
// sl_streaming) along one axis, for a population moving s mean node spacings
// per step: cells of p intervals; node k of a cell (k < p) departs from
// r = xg_k - s / p cells past its cell's start, xg_k = (1 - cos(pi k / p)) / 2,
// which lies in the cell floor(r) cells on, at eta = r - floor(r); its value
// is sum_t psi_t(eta) f(node t of that cell), psi_t the Lagrange polynomials
// through the cell's p + 1 points.  Out: the window offset dmin p (dmin the
// lowest floor(r) over the phases); per phase k, the window weights
// W[k][0..2p] (the phase's p + 1 weights from node b_k = (floor(r_k) -
// dmin) p, zero elsewhere) and the compact entry X[k] = {b_k, psi_0..psi_p,
// 0, 0}.  The weights of each phase are quantized to sum to one (bits as in
// quantize_unit_sum).  Returns false if the phases span more than two cells.
bool glc_axis(double s, int p, int bits, int* off, double* W, double* X) {
  const double pi = 3.14159265358979323846;
  auto xg = [&](int m) { return 0.5 * (1.0 - std::cos(pi * double(m) / double(p))); };
  int d[8];
  double psi[8][8];
  int dmin = 1 << 30, dmax = -(1 << 30);
  for (int k = 0; k < p; ++k) {
    const double r = xg(k) - s / double(p);
    const double fl = std::floor(r);
    const double eta = r - fl;
    d[k] = int(fl);
    dmin = std::min(dmin, d[k]);
    dmax = std::max(dmax, d[k]);
    for (int t = 0; t <= p; ++t) {
      double num = 1.0, den = 1.0;
      for (int m = 0; m <= p; ++m) {
        if (m == t) continue;
        num *= eta - xg(m);
        den *= xg(t) - xg(m);
      }
      psi[k][t] = num / den;
    }
    quantize_unit_sum(psi[k], p + 1, bits);
  }
  if (dmax > dmin + 1) return false;
  *off = dmin * p;
  const int win = 2 * p + 1;
  for (int k = 0; k < p; ++k) {
    const int b = (d[k] - dmin) * p;
    for (int u = 0; u < win; ++u) W[k * win + u] = 0.0;
    for (int u = 0; u < 8; ++u) X[k * 8 + u] = 0.0;
    X[k * 8] = double(b);
    for (int t = 0; t <= p; ++t) {
      W[k * win + b + t] = psi[k][t];
      X[k * 8 + 1 + t] = psi[k][t];
    }
  }
  return true;
}

}  // namespace

struct lbm_ctx {
  int set = 0, D = 0, Q = 0, A = 1, order = 2, ns_user = 4, ns = 4, storage = LBM_F32;
  int degree = 0;
  int64_t n[3] = {1, 1, 1};
  int bc[3] = {0, 0, 0};
  int64_t ncell = 0;
  double tau = 1.0, dx = 1.0, dt = 1.0, cs = 0.0, cs_tab = 0.0, gamma = 1.4;
  int e64 = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  void* buf[2] = {nullptr, nullptr};
  int cur = 0;
  size_t elem = 4, state_bytes = 0;
  Kernels k;
  int* d_off = nullptr;
  void* d_wts = nullptr;
  int* d_off_t = nullptr;
  void* d_wts_t = nullptr;
  void* d_glcx = nullptr;   // cell-wise support: compact per-phase entries [Q][3][p][8]
  int glc_p = 0;            // cell-wise support: cell order p (0: uniform support)
  int cus = 0;              // compute units of the device
  double prandtl = 1.0;     // compressible model: Prandtl number (1: plain BGK)
  int rounding = LBM_ROUND_NEAREST;  // how 16-bit storage rounds
  uint32_t seed = 0;        // stochastic rounding: seed of the random bits
  uint64_t nstep = 0;       // steps the context has taken (stochastic rounding's counter)
  double* d_partial = nullptr;
  double* d_result = nullptr;
  double* h_result = nullptr;
  void* scratch = nullptr;  // device address of the static scratch on `device`
  bool onlattice = false;
  double sw = 0, swx[3] = {0, 0, 0}, swX = 0;
};

namespace {

size_t elem_size(int storage) {
  switch (storage) {
  case LBM_F64: return 8;
  case LBM_F32: return 4;
  case LBM_BF16DEV: return 2;
  case LBM_F16DEV: return 2;
  default: return 0;
  }
}

bool compute_is_f64(const lbm_ctx* c) { return c->storage == LBM_F64; }

int check_ctx(const lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "null context");
  return LBM_OK;
}

int set_device(const lbm_ctx* c) {
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return LBM_OK;
}

// 1 / sum_i w_i xh_ix^2 - 1 with the weights and abscissae rounded to float,
// the compute type of the deviation forms (unused by the FP64 form).  The sets
// are symmetric under exchange of axes, so one axis gives the factor.
double momentum_norm(const lbm_ctx* c) {
  if (compute_is_f64(c)) return 0.0;
  const SetTable t = set_table(c->set);
  double s = 0.0;
  for (int i = 0; i < t.Q; ++i) {
    const double x = double(float(t.xh[i][0]));
    s += double(float(t.w[i])) * x * x;
  }
  return 1.0 / s - 1.0;
}

// Moment defects of the FP32-rounded set (weights, abscissae and |xh|^2 as
// the kernels round them) against the Gaussian moments, in the layout of
// KParams::mdef.
void float_moment_defects(int set, double* out) {
  const SetTable t = set_table(set);
  const int D = t.D;
  // exponents of the monomials (x, y, z) and their multiplicities
  static const int quad[6][3] = {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}};
  static const double quad_mult[6] = {1, 1, 1, 2, 2, 2};
  static const int quart[15][3] = {{4, 0, 0}, {0, 4, 0}, {0, 0, 4}, {3, 1, 0}, {3, 0, 1}, {1, 3, 0}, {0, 3, 1},
                                   {1, 0, 3}, {0, 1, 3}, {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1}, {1, 2, 1},
                                   {1, 1, 2}};
  static const double quart_mult[15] = {1, 1, 1, 4, 4, 4, 4, 4, 4, 6, 6, 6, 12, 12, 12};
  // Gaussian moment E[x^a y^b z^c] with unit variance: product of (k-1)!! for even k
  auto gauss = [&](const int* e) {
    double g = 1.0;
    for (int a = 0; a < 3; ++a) {
      if (e[a] && a >= D) return 0.0;
      if (e[a] % 2) return 0.0;
      for (int k = e[a] - 1; k > 1; k -= 2) g *= k;
    }
    return g;
  };
  auto unused = [&](const int* e) {
    for (int a = D; a < 3; ++a)
      if (e[a]) return true;
    return false;
  };
  double m0 = 0, mX = 0, mXX = 0, m2[6] = {0, 0, 0, 0, 0, 0}, mX2[6] = {0, 0, 0, 0, 0, 0};
  double m4[15] = {0};
  for (int i = 0; i < t.Q; ++i) {
    const double w = double(float(t.w[i]));
    double xe = 0;
    for (int a = 0; a < 3; ++a) xe += t.xh[i][a] * t.xh[i][a];
    const double X = double(float(xe));
    double x[3];
    for (int a = 0; a < 3; ++a) x[a] = double(float(t.xh[i][a]));
    auto mono = [&](const int* e) {
      double v = 1.0;
      for (int a = 0; a < 3; ++a)
        for (int k = 0; k < e[a]; ++k) v *= x[a];
      return v;
    };
    m0 += w;
    mX += w * X;
    mXX += w * X * X;
    for (int k = 0; k < 6; ++k) {
      m2[k] += w * mono(quad[k]);
      mX2[k] += w * X * mono(quad[k]);
    }
    for (int k = 0; k < 15; ++k) m4[k] += w * mono(quart[k]);
  }
  for (int k = 0; k < MDEF_N; ++k) out[k] = 0.0;
  out[0] = m0 - 1.0;
  out[7] = mX - D;
  out[14] = mXX - double(D * (D + 2));
  for (int k = 0; k < 6; ++k) {
    if (unused(quad[k])) continue;
    out[1 + k] = quad_mult[k] * (m2[k] - gauss(quad[k]));
    out[8 + k] = quad_mult[k] * (mX2[k] - (D + 2) * gauss(quad[k]));
  }
  for (int k = 0; k < 15; ++k) {
    if (unused(quart[k])) continue;
    out[15 + k] = quart_mult[k] * (m4[k] - gauss(quart[k]));
  }
}

void mass_defects(const lbm_ctx* c, double* out) {
  if (compute_is_f64(c)) {
    for (int k = 0; k < MDEF_N; ++k) out[k] = 0.0;
    return;
  }
  float_moment_defects(c->set, out);
}

KParams base_params(const lbm_ctx* c) {
  KParams p{};
  p.off = c->d_off;
  p.wts = c->d_wts;
  p.off_t = c->d_off_t;
  p.wts_t = c->d_wts_t;
  p.glcx = c->d_glcx;
  p.cus = c->cus;
  p.inv_pr = 1.0 / c->prandtl;
  for (int a = 0; a < 3; ++a) {
    p.n[a] = int(c->n[a]);
    p.bc[a] = c->bc[a];
  }
  p.pstride = c->ncell;
  p.omega = 1.0 / c->tau;
  p.tau_m_half = c->tau - 0.5;
  const double Cv = c->A == 2 ? 1.0 / (c->gamma - 1.0) : 0.5 * c->D;
  p.cv2mD = 2.0 * Cv - c->D;
  p.inv2cv = 1.0 / (2.0 * Cv);
  p.sw = c->sw;
  for (int a = 0; a < 3; ++a) p.swx[a] = c->swx[a];
  p.swX = c->swX;
  p.e64 = c->e64 ? 1.0 : 0.0;
  p.cmom1 = momentum_norm(c);
  mass_defects(c, p.mdef);
  return p;
}

CellParams base_cell(const lbm_ctx* c) {
  CellParams p{};
  p.ncell = c->ncell;
  p.cs = c->cs;
  const double Cv = c->A == 2 ? 1.0 / (c->gamma - 1.0) : 0.5 * c->D;
  p.cv2mD = 2.0 * Cv - c->D;
  p.inv2cv = 1.0 / (2.0 * Cv);
  p.sw = c->sw;
  p.swX = c->swX;
  for (int a = 0; a < 3; ++a) p.swx[a] = c->swx[a];
  p.scale = 1.0 / double(c->ncell);
  return p;
}

// Host stencil tables for the kernels: offsets [Q][3] and weights [Q][3][ns]
// in the compute type; `transpose` gives the stencil of S^T (mirrored offsets,
// reversed weights).
// Cell-wise support (glc_p > 0): offsets [Q][3] (the window's start, dmin p
// nodes from the arrival node's cell), window weights w [Q][3][p][2p + 1] and
// compact entries x [Q][3][p][8] (glc_axis); axes along which a population
// does not move keep offset 0 and are never interpolated.  Returns false if
// some population's phases span more than two cells.
bool build_glc_tables(const lbm_ctx* c, std::vector<int>& off, std::vector<double>& w, std::vector<double>& x) {
  const SetTable t = set_table(c->set);
  const int p = c->glc_p, win = 2 * p + 1;
  off.assign(size_t(c->Q) * 3, 0);
  w.assign(size_t(c->Q) * 3 * p * win, 0.0);
  x.assign(size_t(c->Q) * 3 * p * 8, 0.0);
  const int bits = compute_is_f64(c) ? 53 : 24;
  for (int i = 0; i < c->Q; ++i)
    for (int a = 0; a < c->D; ++a) {
      if (t.xh[i][a] == 0.0) continue;
      const double s = t.xh[i][a] * c->cs * c->dt / c->dx;
      if (!glc_axis(s, p, bits, &off[i * 3 + a], &w[(size_t(i) * 3 + a) * p * win], &x[(size_t(i) * 3 + a) * p * 8]))
        return false;
    }
  return true;
}

void build_tables(const lbm_ctx* c, bool transpose, std::vector<int>& off, std::vector<double>& w) {
  const SetTable t = set_table(c->set);
  const int ns = c->ns;
  off.assign(size_t(c->Q) * 3, 0);
  w.assign(size_t(c->Q) * 3 * ns, 0.0);
  const int bits = compute_is_f64(c) ? 53 : 24;
  for (int i = 0; i < c->Q; ++i)
    for (int a = 0; a < 3; ++a) {
      double* L = &w[(size_t(i) * 3 + a) * ns];
      if (a >= c->D || t.xh[i][a] == 0.0) {
        off[i * 3 + a] = 0;
        L[0] = 1.0;
        continue;
      }
      const double s = t.xh[i][a] * c->cs * c->dt / c->dx;
      int first = 0;
      double Lt[MAXNS] = {0, 0, 0, 0, 0};
      int taps = ns;
      if (c->onlattice || c->ns_user == 1) {
        // one node: the departure node itself (integer shift) or the nearest one
        stencil_axis(s, 1, &first, Lt);
        taps = 1;
      } else {
        stencil_axis(s, ns, &first, Lt);
        quantize_unit_sum(Lt, ns, bits);
      }
      if (transpose) {
        // (S^T v)(y) = sum_k L_k v(y - first - k): first node -first - (taps-1), weights reversed
        off[i * 3 + a] = -first - (taps - 1);
        for (int k = 0; k < taps; ++k) L[k] = Lt[taps - 1 - k];
      } else {
        off[i * 3 + a] = first;
        for (int k = 0; k < taps; ++k) L[k] = Lt[k];
      }
    }
}

// The kernels wrap a periodic node index i with one add or subtract, valid
// for -N <= i < 2N; the nodes of a stencil run from j + o to j + o + n - 1
// for arrival nodes 0 <= j < N, so every offset o needs -N <= o and
// o + n <= N + 1.
int check_reach(const lbm_ctx* c) {
  if (c->glc_p) {
    // the window of a tile runs from its first cell's start + dmin p to its last
    // cell's start + (dmin + 2) p; the kernels wrap indices in [-N, 2N)
    std::vector<int> off;
    std::vector<double> w, x;
    if (!build_glc_tables(c, off, w, x)) return fail(LBM_EINVAL, "a population's phases span more than two cells");
    for (int i = 0; i < c->Q; ++i)
      for (int a = 0; a < c->D; ++a) {
        const int64_t o = off[i * 3 + a], N = c->n[a];
        if (o < -N || o + 2 * c->glc_p > N)
          return fail(LBM_EINVAL, "grid extent " + std::to_string(N) + " along axis " + std::to_string(a) +
                                      " cannot hold a cell-wise window at offset " + std::to_string(o));
      }
    return LBM_OK;
  }
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<int> off;
    std::vector<double> w;
    build_tables(c, tr == 1, off, w);
    for (int i = 0; i < c->Q; ++i)
      for (int a = 0; a < c->D; ++a) {
        const int64_t o = off[i * 3 + a], N = c->n[a];
        if (c->bc[a] == LBM_PERIODIC && (o < -N || o + c->ns > N + 1))
          return fail(LBM_EINVAL, "grid extent " + std::to_string(N) + " along axis " + std::to_string(a) +
                                      " cannot hold a stencil offset of " + std::to_string(o) + " with " +
                                      std::to_string(c->ns) + " nodes");
      }
  }
  return LBM_OK;
}

// Copies a table of doubles to a new device buffer in the compute type.
int upload_reals(const lbm_ctx* c, const std::vector<double>& v, void** dst, const char* what) {
  const size_t el = compute_is_f64(c) ? sizeof(double) : sizeof(float);
  hipError_t e = hipMalloc(dst, v.size() * el);
  if (e != hipSuccess) return fail(LBM_ENOMEM, std::string("hipMalloc ") + what);
  if (compute_is_f64(c)) {
    e = hipMemcpy(*dst, v.data(), v.size() * el, hipMemcpyHostToDevice);
  } else {
    std::vector<float> f(v.begin(), v.end());
    e = hipMemcpy(*dst, f.data(), f.size() * el, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, what);
  return LBM_OK;
}

int upload_tables(lbm_ctx* c) {
  if (c->glc_p) {
    std::vector<int> off;
    std::vector<double> w, x;
    if (!build_glc_tables(c, off, w, x)) return fail(LBM_EINVAL, "a population's phases span more than two cells");
    hipError_t e = hipMalloc(&c->d_off, off.size() * sizeof(int));
    if (e != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc offsets");
    e = hipMemcpy(c->d_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy offsets");
    if (int r = upload_reals(c, w, &c->d_wts, "window weights")) return r;
    return upload_reals(c, x, &c->d_glcx, "compact weights");
  }
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<int> off;
    std::vector<double> w;
    build_tables(c, tr == 1, off, w);
    int** doff = tr ? &c->d_off_t : &c->d_off;
    void** dw = tr ? &c->d_wts_t : &c->d_wts;
    hipError_t e = hipMalloc(doff, off.size() * sizeof(int));
    if (e != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc offsets");
    e = hipMemcpy(*doff, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy offsets");
    if (compute_is_f64(c)) {
      e = hipMalloc(dw, w.size() * sizeof(double));
      if (e != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc weights");
      e = hipMemcpy(*dw, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice);
    } else {
      std::vector<float> wf(w.begin(), w.end());
      e = hipMalloc(dw, wf.size() * sizeof(float));
      if (e != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc weights");
      e = hipMemcpy(*dw, wf.data(), wf.size() * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy weights");
  }
  return LBM_OK;
}

void release(lbm_ctx* c) {
  if (c->d_off) (void)hipFree(c->d_off);
  if (c->d_wts) (void)hipFree(c->d_wts);
  if (c->d_off_t) (void)hipFree(c->d_off_t);
  if (c->d_wts_t) (void)hipFree(c->d_wts_t);
  if (c->d_glcx) (void)hipFree(c->d_glcx);
  if (c->d_partial) (void)hipFree(c->d_partial);
  if (c->d_result) (void)hipFree(c->d_result);
  if (c->h_result) (void)hipHostFree(c->h_result);
}

int launch(hipError_t e, const char* what) { return e == hipSuccess ? LBM_OK : hip_fail(e, what); }

}  // namespace

extern "C" {

int32_t lbm_abi_version(void) { return 3; }

const char* lbm_strerror(int status) {
  switch (status) {
  case LBM_OK: return "ok";
  case LBM_EINVAL: return "invalid argument";
  case LBM_ENOMEM: return "out of memory";
  case LBM_EHIP: return "HIP runtime error";
  case LBM_EUNSUPPORTED: return "unsupported combination";
  case LBM_EDIVERGED: return "state diverged";
  default: return "unknown status";
  }
}

const char* lbm_last_error(void) { return g_last_error.c_str(); }

void lbm_default_options(lbm_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->storage = LBM_F32;
  opt->stencil = 4;
  opt->dx = 1.0;
  opt->dt = 1.0;
  opt->cs = 0.0;
  opt->gamma = 1.4;
  opt->prandtl = 1.0;
}

int lbm_set_table(int32_t set, int32_t* Q, int32_t* D, int32_t* degree, double* cs, double* w, double* xi) {
  if (set < 0 || set >= NUM_SETS) return fail(LBM_EINVAL, "unknown velocity set");
  if (!Q || !D || !degree || !cs || !w || !xi) return fail(LBM_EINVAL, "null pointer");
  const SetTable t = set_table(set);
  *Q = t.Q;
  *D = t.D;
  *degree = t.degree;
  *cs = t.cs;
  for (int i = 0; i < t.Q; ++i) {
    w[i] = t.w[i];
    for (int a = 0; a < 3; ++a) xi[3 * i + a] = t.xh[i][a] * t.cs;
  }
  return LBM_OK;
}

int lbm_float_moment_defects(int32_t set, double* out) {
  if (set < 0 || set >= NUM_SETS) return fail(LBM_EINVAL, "unknown velocity set");
  if (!out) return fail(LBM_EINVAL, "null pointer");
  float_moment_defects(set, out);
  return LBM_OK;
}

int lbm_stencil(int32_t set, double dt, double dx, double cs, int32_t n, int32_t* offsets, double* weights) {
  if (set < 0 || set >= NUM_SETS) return fail(LBM_EINVAL, "unknown velocity set");
  if (n < 1 || n > MAXNS) return fail(LBM_EINVAL, "stencil length must be 1..5");
  if (!(dt > 0) || !(dx > 0)) return fail(LBM_EINVAL, "dt and dx must be positive");
  if (!offsets || !weights) return fail(LBM_EINVAL, "null pointer");
  const SetTable t = set_table(set);
  const double c = cs > 0 ? cs : t.cs;
  for (int i = 0; i < t.Q; ++i)
    for (int a = 0; a < 3; ++a) {
      double* L = weights + (size_t(i) * 3 + a) * n;
      for (int k = 0; k < n; ++k) L[k] = 0.0;
      if (a >= t.D || t.xh[i][a] == 0.0) {
        offsets[3 * i + a] = 0;
        L[0] = 1.0;
        continue;
      }
      int first = 0;
      double Lt[MAXNS];
      stencil_axis(t.xh[i][a] * c * dt / dx, n, &first, Lt);
      offsets[3 * i + a] = first;
      for (int k = 0; k < n; ++k) L[k] = Lt[k];
    }
  return LBM_OK;
}

int lbm_create(lbm_ctx** out, int32_t set, const int64_t grid[3], double tau, int32_t order, const lbm_options* opt) {
  if (!out) return fail(LBM_EINVAL, "null output pointer");
  *out = nullptr;
  if (set < 0 || set >= NUM_SETS) return fail(LBM_EINVAL, "unknown velocity set");
  if (!grid) return fail(LBM_EINVAL, "null grid");
  lbm_options o;
  if (opt) o = *opt;
  else lbm_default_options(&o);
  const SetTable t = set_table(set);
  auto c = new (std::nothrow) lbm_ctx;
  if (!c) return fail(LBM_ENOMEM, "context allocation");
  c->set = set;
  c->D = t.D;
  c->Q = t.Q;
  c->degree = t.degree;
  c->cs_tab = t.cs;
  auto bad = [&](int code, const std::string& m) {
    release(c);
    delete c;
    return fail(code, m);
  };
  for (int a = 0; a < 3; ++a) {
    c->n[a] = grid[a];
    if (grid[a] < 1) return bad(LBM_EINVAL, "every grid extent must be >= 1");
  }
  if (c->D == 2 && grid[2] != 1) return bad(LBM_EINVAL, "2D sets need nz = 1");
  if (grid[0] > (1 << 30) || grid[1] > (1 << 30) || grid[2] > (1 << 30))
    return bad(LBM_EINVAL, "grid extent too large");
  c->ncell = grid[0] * grid[1] * grid[2];
  if (c->ncell >= (int64_t(1) << 31)) return bad(LBM_EINVAL, "more than 2^31 - 1 cells");
  if (!(tau > 0.5) || !std::isfinite(tau)) return bad(LBM_EINVAL, "tau must exceed 1/2");
  c->tau = tau;
  if (order < 2 || order > 4) return bad(LBM_EINVAL, "order must be 2, 3 or 4");
  if (2 * order > t.degree) return bad(LBM_EUNSUPPORTED, "order too high for the set's degree (need 2N <= d)");
  c->order = order;
  if (o.storage < LBM_F64 || o.storage > LBM_F16DEV) return bad(LBM_EINVAL, "unknown storage");
  c->storage = o.storage;
  c->elem = elem_size(o.storage);
  if (o.stencil < 1 || o.stencil > MAXNS) return bad(LBM_EINVAL, "stencil length must be 1..5");
  c->ns_user = o.stencil;
  if (!(o.dx > 0) || !(o.dt > 0) || !std::isfinite(o.dx) || !std::isfinite(o.dt))
    return bad(LBM_EINVAL, "dx and dt must be positive");
  c->dx = o.dx;
  c->dt = o.dt;
  c->cs = o.cs > 0 ? o.cs : t.cs;
  c->A = o.compressible ? 2 : 1;
  c->gamma = o.gamma;
  if (c->A == 2 && !(o.gamma > 1.0)) return bad(LBM_EINVAL, "gamma must exceed 1");
  c->e64 = o.energy_f64 ? 1 : 0;
  if (c->e64 && (c->A != 2 || (o.storage != LBM_BF16DEV && o.storage != LBM_F16DEV)))
    return bad(LBM_EUNSUPPORTED, "energy_f64 applies to the compressible model with 16-bit storage");
  for (int a = 0; a < 3; ++a) {
    if (o.boundary[a] != LBM_PERIODIC && o.boundary[a] != LBM_EXTRAPOLATE) return bad(LBM_EINVAL, "unknown boundary");
    c->bc[a] = (a < c->D) ? o.boundary[a] : LBM_PERIODIC;
  }
  c->stream = static_cast<hipStream_t>(o.stream);
  // kernels address one population with 32-bit byte offsets, and a partial
  // tile's dropped stores sit one population beyond its start plus at most
  // one xy plane
  if ((size_t(c->ncell) + size_t(grid[0] * grid[1])) * c->elem >= (size_t(1) << 32))
    return bad(LBM_EINVAL, "one population (plus one xy plane) exceeds 4 GiB");
  c->state_bytes = size_t(c->A) * c->Q * size_t(c->ncell) * c->elem;

  // on-lattice: every moving component shifts by a whole number of cells
  bool integral = true;
  for (int i = 0; i < t.Q; ++i)
    for (int a = 0; a < t.D; ++a) {
      if (t.xh[i][a] == 0.0) continue;
      const double s = t.xh[i][a] * c->cs * c->dt / c->dx;
      if (s != std::nearbyint(s)) integral = false;
    }
  // kernel stencil length: on-lattice sets with a copy kernel use one node;
  // the cell-wise support has its own kernels (p = stencil - 1)
  const bool has_copy = (set == LBM_D2Q9 || set == LBM_D3Q27);
  if (o.support != LBM_UNIFORM && o.support != LBM_GLC) return bad(LBM_EINVAL, "unknown streaming support");
  if (o.support == LBM_GLC) {
    c->glc_p = c->ns_user - 1;
    if (c->glc_p != 4) return bad(LBM_EUNSUPPORTED, "cell-wise support is built for p = 4 (stencil 5)");
    for (int a = 0; a < c->D; ++a) {
      if (c->bc[a] != LBM_PERIODIC) return bad(LBM_EUNSUPPORTED, "cell-wise support needs periodic axes");
      if (c->n[a] % c->glc_p) return bad(LBM_EINVAL, "cell-wise support: extents must be multiples of p");
    }
    c->ns = GLC_BASE + c->glc_p;
  } else if ((integral || c->ns_user == 1) && has_copy) {
    c->ns = 1;
    c->onlattice = integral;
  } else if (c->ns_user == 1) {
    c->ns = 2;  // one node, padded with a zero weight
  } else {
    c->ns = c->ns_user;
  }
  if (!find_kernels(set, c->ns, order, c->A, c->storage, &c->k))
    return bad(LBM_EUNSUPPORTED, "no kernel built for this set / stencil / order / model / storage");
  if (o.rounding != LBM_ROUND_NEAREST && o.rounding != LBM_ROUND_STOCHASTIC) return bad(LBM_EINVAL, "unknown rounding");
  if (o.rounding == LBM_ROUND_STOCHASTIC && c->storage != LBM_BF16DEV && c->storage != LBM_F16DEV)
    return bad(LBM_EUNSUPPORTED, "stochastic rounding applies to 16-bit storage");
  c->rounding = o.rounding;
  c->seed = o.seed;
  if (!(o.prandtl > 0) || !std::isfinite(o.prandtl)) return bad(LBM_EINVAL, "the Prandtl number must be positive");
  c->prandtl = o.prandtl;
  if (c->prandtl != 1.0 && !c->k.step_qe)
    return bad(LBM_EUNSUPPORTED, "Pr != 1 is built for the compressible D3Q45 (n = 4) and D2Q19 / D2Q25 (n = 5) "
                                 "models with FP64 / FP32 storage");

  // sums of the stored table (reference values of the deviation storage)
  for (int i = 0; i < t.Q; ++i) {
    c->sw += t.w[i];
    double X = 0;
    for (int a = 0; a < 3; ++a) {
      c->swx[a] += t.w[i] * t.xh[i][a];
      X += t.xh[i][a] * t.xh[i][a];
    }
    c->swX += t.w[i] * X;
  }

  if (check_reach(c) != LBM_OK) return bad(LBM_EINVAL, g_last_error);

  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device);
  if (e != hipSuccess) {
    int r = hip_fail(e, "hipGetDevice");
    release(c);
    delete c;
    return r;
  }
  int rc = upload_tables(c);
  if (rc != LBM_OK) {
    std::string m = g_last_error;
    release(c);
    delete c;
    return fail(rc, m);
  }
  rc = scratch_address(c->device, &c->scratch);
  if (rc != LBM_OK) {
    std::string m = g_last_error;
    release(c);
    delete c;
    return fail(rc, m);
  }
  if (hipMalloc(&c->d_partial, sizeof(double) * MOMENT_BLOCKS * NPART) != hipSuccess ||
      hipMalloc(&c->d_result, sizeof(double) * NPART) != hipSuccess ||
      hipHostMalloc(&c->h_result, sizeof(double) * NPART, hipHostMallocDefault) != hipSuccess)
    return bad(LBM_ENOMEM, "reduction scratch");
  *out = c;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  release(c);
  delete c;
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* c) { return c ? c->state_bytes : 0; }

int lbm_bind(lbm_ctx* c, void* b0, void* b1) {
  if (int r = check_ctx(c)) return r;
  if (!b0 || !b1) return fail(LBM_EINVAL, "null buffer");
  const char* p0 = static_cast<const char*>(b0);
  const char* p1 = static_cast<const char*>(b1);
  if (p0 < p1 + c->state_bytes && p1 < p0 + c->state_bytes) return fail(LBM_EINVAL, "buffers overlap");
  c->buf[0] = b0;
  c->buf[1] = b1;
  c->cur = 0;
  return LBM_OK;
}

void* lbm_state(lbm_ctx* c) { return c ? c->buf[c->cur] : nullptr; }

int lbm_set_stream(lbm_ctx* c, void* stream) {
  if (int r = check_ctx(c)) return r;
  c->stream = static_cast<hipStream_t>(stream);
  return LBM_OK;
}

int lbm_enstrophy(lbm_ctx* c, const void* u, int32_t order, double* enstrophy) {
  if (int r = check_ctx(c)) return r;
  if (!u || !enstrophy) return fail(LBM_EINVAL, "null pointer");
  if (order != 2 && order != 4 && order != 6 && order != 8) return fail(LBM_EINVAL, "order must be 2, 4, 6 or 8");
  for (int a = 0; a < c->D; ++a)
    if (c->bc[a] != LBM_PERIODIC) return fail(LBM_EUNSUPPORTED, "enstrophy needs periodic axes");
  if (int r = set_device(c)) return r;
  // central-difference coefficients of order 2m over the spacing:
  // c_j = (-1)^(j+1) (m!)^2 / (j (m-j)! (m+j)!) / dx
  const int m = order / 2;
  double coef[4];
  auto fact = [](int k) { double f = 1; for (int i = 2; i <= k; ++i) f *= i; return f; };
  for (int j = 1; j <= m; ++j)
    coef[j - 1] = ((j % 2) ? 1.0 : -1.0) * fact(m) * fact(m) / (double(j) * fact(m - j) * fact(m + j)) / c->dx;
  hipError_t e = launch_enstrophy(u, c->storage == LBM_F64, c->n, c->D, m, coef, c->d_partial,
                                  MOMENT_BLOCKS * NPART, c->d_result, c->stream);
  if (e != hipSuccess) return hip_fail(e, "enstrophy kernel");
  e = hipMemcpyAsync(c->h_result, c->d_result, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  *enstrophy = c->h_result[0] / double(c->ncell);
  return LBM_OK;
}

int lbm_sync(lbm_ctx* c) {
  if (int r = check_ctx(c)) return r;
  if (int r = set_device(c)) return r;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "asynchronous error");
  return LBM_OK;
}

int lbm_init_equilibrium(lbm_ctx* c, const void* rho, const void* u, const void* theta) {
  if (int r = check_ctx(c)) return r;
  if (!c->buf[0]) return fail(LBM_EINVAL, "no buffers bound");
  if (!rho || !u) return fail(LBM_EINVAL, "null rho or u");
  if (int r = set_device(c)) return r;
  CellParams p = base_cell(c);
  p.rho = rho;
  p.u = u;
  p.theta = theta;
  p.out_f = c->buf[c->cur];
  return launch(c->k.init(p, c->stream), "init kernel");
}

// Stream-ordered copy of the whole current state; waits for it so that a
// host buffer is complete (or reusable) when the call returns.
static int copy_state(lbm_ctx* c, void* dst, const void* src, const char* what) {
  hipError_t e = hipMemcpyAsync(dst, src, c->state_bytes, hipMemcpyDefault, c->stream);
  if (e != hipSuccess) return hip_fail(e, what);
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return LBM_OK;
}

int lbm_get_state(lbm_ctx* c, void* dst) {
  if (int r = check_ctx(c)) return r;
  if (!c->buf[0]) return fail(LBM_EINVAL, "no buffers bound");
  if (!dst) return fail(LBM_EINVAL, "null destination");
  if (int r = set_device(c)) return r;
  return copy_state(c, dst, c->buf[c->cur], "hipMemcpyAsync (get state)");
}

int lbm_set_state(lbm_ctx* c, const void* src) {
  if (int r = check_ctx(c)) return r;
  if (!c->buf[0]) return fail(LBM_EINVAL, "no buffers bound");
  if (!src) return fail(LBM_EINVAL, "null source");
  if (int r = set_device(c)) return r;
  return copy_state(c, c->buf[c->cur], src, "hipMemcpyAsync (set state)");
}

// MI355X's last-level (Infinity) cache.  While both state buffers fit in it,
// the step's output stays there for the next step's reads; beyond it, the
// output is streamed past the caches (non-temporal stores), leaving them to
// the halo rows that neighbouring tiles re-read.
constexpr size_t LLC_BYTES = size_t(256) << 20;

// Per-step seed of stochastic rounding: the context's seed and step count
// through SplitMix64's finalizer (a published 64-bit mixer).
static uint32_t step_seed(uint32_t seed, uint64_t step) {
  uint64_t z = (uint64_t(seed) << 32 | (step & 0xffffffffu)) + 0x9e3779b97f4a7c15ull * (step >> 32);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return uint32_t((z ^ (z >> 31)) >> 32);
}

static int step_once(lbm_ctx* c, const void* src, void* dst) {
  KParams p = base_params(c);
  p.src = src;
  p.dst = dst;
  p.sr = c->rounding == LBM_ROUND_STOCHASTIC ? 1 : 0;
  p.seed = step_seed(c->seed, c->nstep++);
  const bool big = 2 * c->state_bytes > LLC_BYTES;
  StepLaunch f = (c->k.step_stream && big) ? c->k.step_stream : c->k.mode[MODE_STEP];
  if (c->prandtl != 1.0) f = (c->k.step_qe_stream && big) ? c->k.step_qe_stream : c->k.step_qe;
  return launch(f(p, c->stream), "step kernel");
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (int r = check_ctx(c)) return r;
  if (n < 0) return fail(LBM_EINVAL, "negative step count");
  if (n == 0) return LBM_OK;
  if (!c->buf[0]) return fail(LBM_EINVAL, "no buffers bound");
  if (int r = set_device(c)) return r;
  for (int64_t s = 0; s < n; ++s) {
    if (int r = step_once(c, c->buf[c->cur], c->buf[c->cur ^ 1])) return r;
    c->cur ^= 1;
  }
  return LBM_OK;
}

int lbm_step_into(lbm_ctx* c, const void* src, void* dst) {
  if (int r = check_ctx(c)) return r;
  if (!src || !dst) return fail(LBM_EINVAL, "null buffer");
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  if (a < b + c->state_bytes && b < a + c->state_bytes) return fail(LBM_EINVAL, "src and dst overlap");
  if (int r = set_device(c)) return r;
  return step_once(c, src, dst);
}

// The moments kernel's block sums into `partial` ([nblocks][NPART]), their
// sum into `result` ([NPART]), copied to the host array `host` ([NPART]);
// waits for the stream.
static int moments_impl(lbm_ctx* c, const void* state, void* rho, void* u, void* theta, lbm_diag* diag,
                        double* partial, double* result, double* host) {
  CellParams p = base_cell(c);
  p.f = state;
  p.out_rho = rho;
  p.out_u = u;
  p.out_theta = theta;
  p.partial = partial;
  p.nblocks = moment_blocks(c->ncell);
  if (int r = launch(c->k.moments(p, c->stream), "moments kernel")) return r;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, c->stream, partial, p.nblocks, result);
  if (int r = launch(hipGetLastError(), "reduce kernel")) return r;
  hipError_t e = hipMemcpyAsync(host, result, sizeof(double) * NPART, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  lbm_diag d{};
  d.mass = host[0];
  d.momentum[0] = host[1];
  d.momentum[1] = host[2];
  d.momentum[2] = host[3];
  d.ke = host[4] / double(c->ncell);
  d.energy = host[5];
  d.min_rho = host[6];
  d.min_theta = host[7];
  d.nonfinite = int32_t(host[8]);
  if (diag) *diag = d;
  if (d.nonfinite > 0 || !(d.min_rho > 0) || !(d.min_theta > 0))
    return fail(LBM_EDIVERGED, "non-finite value, rho <= 0 or theta <= 0");
  return LBM_OK;
}

int lbm_moments(lbm_ctx* c, const void* state, void* rho, void* u, void* theta, lbm_diag* diag) {
  if (int r = check_ctx(c)) return r;
  if (!state) state = c->buf[c->cur];
  if (!state) return fail(LBM_EINVAL, "no state");
  if (int r = set_device(c)) return r;
  return moments_impl(c, state, rho, u, theta, diag, c->d_partial, c->d_result, c->h_result);
}

int lbm_moments_noalloc(lbm_ctx* c, const void* state, void* rho, void* u, void* theta, lbm_diag* diag) {
  if (int r = check_ctx(c)) return r;
  if (!state) state = c->buf[c->cur];
  if (!state) return fail(LBM_EINVAL, "no state");
  const size_t need = size_t(moment_blocks(c->ncell) + 1) * NPART;
  if (need > SCRATCH_DOUBLES)
    return fail(LBM_EINVAL, "lbm_moments_noalloc: " + std::to_string(need) + " doubles of reduction scratch exceed " +
                                "the static maximum of " + std::to_string(SCRATCH_DOUBLES));
  if (int r = set_device(c)) return r;
  double* base = static_cast<double*>(c->scratch);
  if (!base) return fail(LBM_EINVAL, "no static scratch address for this context's device");
  double host[NPART];
  return moments_impl(c, state, rho, u, theta, diag, base, base + size_t(moment_blocks(c->ncell)) * NPART, host);
}

static int adjoint_ok(lbm_ctx* c) {
  if (int r = check_ctx(c)) return r;
  if (!c->k.mode[MODE_ADJ_STEP]) return fail(LBM_EUNSUPPORTED, "adjoint needs the weakly compressible model with FP64/FP32");
  for (int a = 0; a < c->D; ++a)
    if (c->bc[a] != LBM_PERIODIC) return fail(LBM_EUNSUPPORTED, "adjoint needs periodic axes");
  return set_device(c);
}

int lbm_adjoint_collide(lbm_ctx* c, const void* f_prev, const void* lam, void* nu) {
  if (int r = adjoint_ok(c)) return r;
  if (!f_prev || !lam || !nu) return fail(LBM_EINVAL, "null buffer");
  KParams p = base_params(c);
  p.src = f_prev;
  p.src2 = lam;
  p.dst = nu;
  return launch(c->k.mode[MODE_ADJ_COLLIDE](p, c->stream), "adjoint collide kernel");
}

int lbm_adjoint_stream(lbm_ctx* c, const void* nu, void* lam) {
  if (int r = adjoint_ok(c)) return r;
  if (!nu || !lam) return fail(LBM_EINVAL, "null buffer");
  if (nu == lam) return fail(LBM_EINVAL, "nu and lam must differ");
  KParams p = base_params(c);
  p.src = nu;
  p.src2 = nu;
  p.dst = lam;
  return launch(c->k.mode[MODE_ADJ_STREAM](p, c->stream), "adjoint stream kernel");
}

int lbm_stream(lbm_ctx* c, const void* src, void* dst) {
  if (int r = adjoint_ok(c)) return r;
  if (!src || !dst) return fail(LBM_EINVAL, "null buffer");
  if (src == dst) return fail(LBM_EINVAL, "src and dst must differ");
  KParams p = base_params(c);
  p.src = src;
  p.src2 = src;
  p.dst = dst;
  // the transposed-streaming kernel with the forward stencil is plain streaming
  p.off_t = c->d_off;
  p.wts_t = c->d_wts;
  return launch(c->k.mode[MODE_ADJ_STREAM](p, c->stream), "stream kernel");
}

int lbm_adjoint_step(lbm_ctx* c, const void* f_prev, const void* nu_in, void* nu_out) {
  if (int r = adjoint_ok(c)) return r;
  if (!f_prev || !nu_in || !nu_out) return fail(LBM_EINVAL, "null buffer");
  if (nu_in == nu_out) return fail(LBM_EINVAL, "nu_in and nu_out must differ");
  KParams p = base_params(c);
  p.src = f_prev;
  p.src2 = nu_in;
  p.dst = nu_out;
  return launch(c->k.mode[MODE_ADJ_STEP](p, c->stream), "adjoint step kernel");
}

int lbm_ke_adjoint(lbm_ctx* c, const void* f, void* lam) {
  if (int r = adjoint_ok(c)) return r;
  if (!f || !lam) return fail(LBM_EINVAL, "null buffer");
  CellParams p = base_cell(c);
  p.f = f;
  p.out_f = lam;
  return launch(c->k.ke_adjoint(p, c->stream), "ke adjoint kernel");
}

int lbm_init_equilibrium_adjoint(lbm_ctx* c, const void* rho, const void* u, const void* lam0, void* grad_u) {
  if (int r = adjoint_ok(c)) return r;
  if (!rho || !u || !lam0 || !grad_u) return fail(LBM_EINVAL, "null buffer");
  CellParams p = base_cell(c);
  p.rho = rho;
  p.u = u;
  p.lam = lam0;
  p.out_u = grad_u;
  return launch(c->k.init_adjoint(p, c->stream), "init adjoint kernel");
}

}  // extern "C"

namespace lbm {

template <int SET, int ST, int NS>
static bool find_part(int order, int arrays, Kernels* out) {
  if constexpr (part_exists<SET, ST, NS>()) return find_kernels_part<SET, ST, NS>(order, arrays, out);
  return false;
}

template <int SET, int ST>
static bool find_st(int ns, int order, int arrays, Kernels* out) {
  switch (ns) {
  case 1: return find_part<SET, ST, 1>(order, arrays, out);
  case 2: return find_part<SET, ST, 2>(order, arrays, out);
  case 3: return find_part<SET, ST, 3>(order, arrays, out);
  case 4: return find_part<SET, ST, 4>(order, arrays, out);
  case 5: return find_part<SET, ST, 5>(order, arrays, out);
  case GLC_P4: return find_part<SET, ST, GLC_P4>(order, arrays, out);
  default: return false;
  }
}

template <int SET>
static bool find_set(int ns, int order, int arrays, int storage, Kernels* out) {
  switch (storage) {
  case ST_F64: return find_st<SET, ST_F64>(ns, order, arrays, out);
  case ST_F32: return find_st<SET, ST_F32>(ns, order, arrays, out);
  case ST_BF16: return find_st<SET, ST_BF16>(ns, order, arrays, out);
  case ST_F16: return find_st<SET, ST_F16>(ns, order, arrays, out);
  default: return false;
  }
}

bool find_kernels(int set, int ns, int order, int arrays, int storage, Kernels* out) {
  switch (set) {
  case D2Q9: return find_set<D2Q9>(ns, order, arrays, storage, out);
  case D2Q19: return find_set<D2Q19>(ns, order, arrays, storage, out);
  case D2Q25: return find_set<D2Q25>(ns, order, arrays, storage, out);
  case D3Q13: return find_set<D3Q13>(ns, order, arrays, storage, out);
  case D3Q21: return find_set<D3Q21>(ns, order, arrays, storage, out);
  case D3Q27: return find_set<D3Q27>(ns, order, arrays, storage, out);
  case D3V27: return find_set<D3V27>(ns, order, arrays, storage, out);
  case D3Q45: return find_set<D3Q45>(ns, order, arrays, storage, out);
  default: return false;
  }
}

}  // namespace lbm
