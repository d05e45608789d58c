// Fused semi-Lagrangian stream + collide kernels for gfx950 (MI355X).
//
// One kernel template serves every velocity set, stencil length, Hermite
// order, storage type and mode (forward step, collision adjoint, fused reverse
// step, transposed streaming).  The set is a template parameter, so every
// population's abscissa is a compile-time constant: zero components drop out
// of the moment and equilibrium arithmetic, and an axis along which a
// population does not move costs neither a halo nor an interpolation pass.
//
// Work decomposition (3D).  A block of NW waves (4; 8 for some sets) owns a
// 64 x NW x RO tile of cells: lane = x, wave = y, and each thread holds RO
// cells along z.  For each population (unrolled at compile time) the block
//   A. loads, per column of the population's source region (the tile shifted
//      by the stencil's first-node offset, widened by n - 1 along every moving
//      axis; x in pairs of adjacent nodes), the RO + n - 1 values along z,
//      interpolates along z in registers and writes RO values per column to
//      LDS;
//   B. interpolates along y in LDS (one thread per (z, x) column);
//   C. interpolates along x from LDS into the thread's registers.
// A population that moves along z only never touches LDS.  The HBM loads of
// the next populations are issued before the current ones are interpolated;
// in 3D two populations share each pair of block barriers.  After the last
// population each thread holds all interpolated populations of its RO cells,
// forms the moments, the Hermite equilibrium in its scalar closed form and
// the BGK update in registers, and stores coalesced along x.
// 2D: the same with y in the role of z and the waves splitting y.
//
// The stencil (first-node offsets and Lagrange weights per population and
// axis) is computed on the host and read through uniform (scalar) loads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "lbm_sets.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// Storage types
// ---------------------------------------------------------------------------

enum Storage : int { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2, ST_F16 = 3 };

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// round to nearest even, NaN stays NaN: gfx950's conversion (one instruction;
// bit-identical to the add-and-truncate form on 5.2 million test values,
// subnormals, ties and specials included)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) { return __builtin_bit_cast(uint16_t, __bf16(f)); }

// Stochastic rounding with random bits rnd: gfx950's conversions, which round
// the magnitude up with probability equal to the dropped fraction of a unit
// in the last place (mean-zero error below one unit; measured: round-up
// frequencies 0.100 / 0.250 / 0.500 / 0.750 / 0.900 at fractions 0.1 ... 0.9
// over 2^20 draws, both signs, FP16 subnormals included).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __fp16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float f, uint32_t rnd) {
  const bf16x2 v = __builtin_amdgcn_cvt_sr_bf16_f32(bf16x2{}, f, rnd, false);
  return __builtin_bit_cast(uint16_t, v[0]);
}
__device__ __forceinline__ _Float16 f32_to_f16_sr(float f, uint32_t rnd) {
  const f16x2 v = __builtin_amdgcn_cvt_sr_f16_f32(f16x2{}, f, rnd, false);
  return __builtin_bit_cast(_Float16, v[0]);
}

// Wellons' 32-bit integer hash ("lowbias32": two multiply-xorshift rounds), the
// random bits of stochastic rounding.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// dev: the kernels compute on deviations d = f - r from the reference values
//      r_i = w_i (f) and (2 C_v - D) w_i (g), which keeps rounding relative to
//      the small deviations instead of the populations;
// stores_dev: the buffer itself holds deviations (all but FP64);
// coarse: 16-bit storage, whose rounding lies far above the FP32 arithmetic's:
//      no energy restoration in the collision; optional FP64 energy sum.
// ldb/stb: buffer accesses at byte offset voff (per lane) + soff (uniform,
// scalar register), so that a row offset shared by the block costs no vector
// instruction.  The resource covers one population array (< 4 GiB).  stb's
// CP is the instruction's cache-policy field: 0, or CP_STREAM (the
// non-temporal bit) for data that no later access of this launch reads.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int CP_STREAM = 2;  // cache policy: non-temporal (streamed) store

// Byte offset of element e for a buffer access, in unsigned 32-bit arithmetic
// (the host keeps every population, plus one xy plane, below 4 GiB).
template <class E>
__device__ __forceinline__ int boff(int e) {
  return int(uint32_t(e) * uint32_t(sizeof(E)));
}
template <class E>
__device__ __forceinline__ rsrc_t make_rsrc(const E* base, int64_t nelem) {
  // word 3 = 0x00020000: raw (unformatted) 32-bit buffer on gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<E*>(base), (short)0, int(uint32_t(nelem * int64_t(sizeof(E)))),
                                           0x00020000);
}

template <int S> struct StoreT;
template <> struct StoreT<ST_F64> {
  using elem = double; using real = double;
  static constexpr bool dev = false, stores_dev = false, coarse = false;
  static __device__ __forceinline__ real ld(const elem* p) { return *p; }
  static __device__ __forceinline__ void st(elem* p, real v) { *p = v; }
  static __device__ __forceinline__ real ldb(rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void stb(real v, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v), r,
                                          voff, soff, CP);
  }
  static __device__ __forceinline__ void ldb2(rsrc_t r, int voff, int soff, real& lo, real& hi) {
    // (elements copied to scalars first: bit-casting a vector element
    // directly reinterprets the vector's first element)
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    const unsigned v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
    lo = __builtin_bit_cast(double, (uint64_t(v1) << 32) | v0);
    hi = __builtin_bit_cast(double, (uint64_t(v3) << 32) | v2);
  }
};
template <> struct StoreT<ST_F32> {
  using elem = float; using real = float;
  static constexpr bool dev = true, stores_dev = true, coarse = false;
  static __device__ __forceinline__ real ld(const elem* p) { return *p; }
  static __device__ __forceinline__ void st(elem* p, real v) { *p = v; }
  static __device__ __forceinline__ real ldb(rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void stb(real v, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, CP);
  }
  static __device__ __forceinline__ void ldb2(rsrc_t r, int voff, int soff, real& lo, real& hi) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    const unsigned v0 = v[0], v1 = v[1];  // scalars first, as above
    lo = __builtin_bit_cast(float, v0);
    hi = __builtin_bit_cast(float, v1);
  }
};
template <> struct StoreT<ST_BF16> {
  using elem = uint16_t; using real = float;
  static constexpr bool dev = true, stores_dev = true, coarse = true;
  static __device__ __forceinline__ real ld(const elem* p) { return bf16_to_f32(*p); }
  static __device__ __forceinline__ void st(elem* p, real v) { *p = f32_to_bf16(v); }
  static __device__ __forceinline__ real ldb(rsrc_t r, int voff, int soff) {
    return bf16_to_f32(__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void stb(real v, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16(v), r, voff, soff, CP);
  }
  // stochastic rounding with random bits rnd
  template <int CP = 0>
  static __device__ __forceinline__ void stb_sr(real v, uint32_t rnd, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b16(f32_to_bf16_sr(v, rnd), r, voff, soff, CP);
  }
  static __device__ __forceinline__ void st_sr(elem* p, real v, uint32_t rnd) { *p = f32_to_bf16_sr(v, rnd); }
  static __device__ __forceinline__ void ldb2(rsrc_t r, int voff, int soff, real& lo, real& hi) {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    lo = bf16_to_f32(uint16_t(v & 0xffffu));
    hi = bf16_to_f32(uint16_t(v >> 16));
  }
};
template <> struct StoreT<ST_F16> {
  using elem = _Float16; using real = float;
  static constexpr bool dev = true, stores_dev = true, coarse = true;
  static __device__ __forceinline__ real ld(const elem* p) { return float(*p); }
  static __device__ __forceinline__ void st(elem* p, real v) { *p = _Float16(v); }
  static __device__ __forceinline__ void st_sr(elem* p, real v, uint32_t rnd) { *p = f32_to_f16_sr(v, rnd); }
  static __device__ __forceinline__ real ldb(rsrc_t r, int voff, int soff) {
    return float(__builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0)));
  }
  template <int CP = 0>
  static __device__ __forceinline__ void stb(real v, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, _Float16(v)), r, voff, soff, CP);
  }
  // stochastic rounding with random bits rnd
  template <int CP = 0>
  static __device__ __forceinline__ void stb_sr(real v, uint32_t rnd, rsrc_t r, int voff, int soff) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, f32_to_f16_sr(v, rnd)), r, voff, soff,
                                          CP);
  }
  static __device__ __forceinline__ void ldb2(rsrc_t r, int voff, int soff, real& lo, real& hi) {
    const unsigned v = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    lo = float(__builtin_bit_cast(_Float16, uint16_t(v & 0xffffu)));
    hi = float(__builtin_bit_cast(_Float16, uint16_t(v >> 16)));
  }
};

// ---------------------------------------------------------------------------
// Compile-time loop
// ---------------------------------------------------------------------------

template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// Kernel parameters
// ---------------------------------------------------------------------------

enum Mode : int {
  MODE_STEP = 0,        // f' = C(S f)
  MODE_ADJ_COLLIDE = 1, // nu = J_C(S f)^T lam
  MODE_ADJ_STEP = 2,    // nu' = J_C(S f)^T (S^T nu)
  MODE_ADJ_STREAM = 3,  // lam = S^T nu
  MODE_STEP_QE = 4      // f' = C(S f), compressible collision with the Pr != 1 quasi-equilibrium
};
constexpr bool is_step(int mode) { return mode == MODE_STEP || mode == MODE_STEP_QE; }

// Streaming supports.  NS <= GLC_BASE: a uniform grid with an NS-node Lagrange
// stencil around the departure point, the same for every node.
// NS = GLC_BASE + p: the paper's cell-wise interpolation (Sec. 3, eq.
// sl_streaming): every axis is cut into cells of p + 1 Gauss-Lobatto-Chebyshev
// support points (neighbouring cells share their end points), and a node's
// departure point is interpolated with the points of the cell that holds it.
// The weights then depend on the node's phase k (its index within its cell,
// 0..p-1) as well as on the population.  Over the p phases the source cells
// are two neighbours at most, so one window of 2p + 1 nodes, starting dmin p
// nodes from the arrival node's cell (dmin the lower source cell's offset),
// serves every phase: the tables hold the window's weights per (population,
// axis, phase), zero outside the phase's own source cell, and a compact form
// (the phase's first window node and its p + 1 weights).
constexpr int GLC_BASE = 16;
template <int NS>
struct Support {
  static constexpr bool glc = NS > GLC_BASE;
  static constexpr int p = glc ? NS - GLC_BASE : 1;  // cell order: phases per axis
  static constexpr int win = glc ? 2 * p + 1 : NS;   // window nodes of one output
  static constexpr int halo = glc ? p + 1 : NS - 1;  // source nodes beyond a tile of whole cells
  static constexpr int xent = 8;                     // compact entry: first node, p + 1 weights, padding
};

struct KParams {
  const void* src;     // populations interpolated with the forward stencil (f)
  const void* src2;    // second input: lam (ADJ_COLLIDE) or nu (ADJ_STEP / ADJ_STREAM)
  void* dst;
  const int* off;      // [Q][3] first-node offsets, forward stencil
  const void* wts;     // [Q][3][NS] weights (compute type), forward stencil;
                       // cell-wise support: [Q][3][p][2p + 1] window weights per phase
  const void* glcx;    // cell-wise support: [Q][3][p][8] compact entries (compute type)
  const int* off_t;    // transposed stencil (adjoint modes)
  const void* wts_t;
  int n[3];            // nx, ny, nz
  int bc[3];           // 0 periodic, 1 extrapolate (clamp)
  int64_t pstride;     // cells per population
  int tiles[3];        // tiles along x, y (3D) / outer (2D), z (3D)
  int chunk;           // tiles per XCD
  int rsy, rsz;        // 3D: y and z tiles of each XCD's block of the grid (0: linear order)
  int ysl;             // 3D: log2 of the XCD blocks along y (1: 2 x 4 (y, z) blocks, 2: 4 x 2)
  int by, bz;          // 3D brick order: bricks of by x bz (y, z) tiles (0: x, y, z order)
  int cus;             // compute units of the device (host input: sizes the brick order)
  double omega;        // 1 / tau (weakly compressible)
  double tau_m_half;   // tau_ref - 1/2 (compressible)
  double cv2mD;        // 2 C_v - D
  double inv2cv;       // 1 / (2 C_v)
  double sw;           // sum_i w_i of the stored table
  double swx[3];       // sum_i w_i xh_i
  double swX;          // sum_i w_i |xh_i|^2
  double e64;          // nonzero: compressible energy moment summed in FP64
  double cmom1;        // 1 / sum_i w_i xh_ix^2 - 1 with the FP32-rounded constants
  double inv_pr;       // MODE_STEP_QE: 1 / Pr
  // FP32 compressible model: defects of the FP32-rounded set's moments against
  // the Gaussian ones (MASS_* layout below), for the mass restoration
  double mdef[30];
  uint32_t seed;       // stochastic rounding: this launch's seed
  int sr;              // nonzero: 16-bit step stores round stochastically (host: selects the RND variant)
};

// Layout of KParams::mdef: [0] sum w - 1; [1..6] quadratic, [8..13]
// |xh|^2-weighted quadratic moments, each times its multiplicity, monomials
// xx yy zz xy xz yz; [7] sum w |xh|^2 - D; [14] sum w |xh|^4 - D(D+2);
// [15..29] quartic moments times multiplicity, monomials xxxx yyyy zzzz
// xxxy xxxz yyyx yyyz zzzx zzzy xxyy xxzz yyzz xxyz yyxz zzxy.
constexpr int MDEF_N = 30;

// Cells per thread along the register (outer) axis: every cell keeps its
// A * Q interpolated values in registers until the collision.
template <int D, int Q, int A, int ST, int MODE>
constexpr int cells_per_thread() {
  constexpr int rb = (ST == ST_F64) ? 8 : 4;
  constexpr int vals = A * Q * (rb / 4) * ((MODE == MODE_ADJ_STEP || MODE == MODE_ADJ_COLLIDE) ? 2 : 1);
  // 2D grids are small (512^2 = 2^18 cells): two cells per thread for the
  // f + g sets keeps more than two blocks per compute unit
  if (D == 2) return vals <= 30 ? 4 : (vals <= 80 ? 2 : 1);
  // FP64 holds a value in two registers
  if (ST == ST_F64) return vals <= 30 ? 4 : (vals <= 60 ? 2 : 1);
  // two cells per thread up to 90 values, the D3Q45 f + g kernels included:
  // fewer halo re-reads, measured faster at 256^3 than one cell per thread at
  // higher occupancy (FP32 5.56 against 7.16 ms)
  return vals <= 30 ? 4 : (vals <= 90 ? 2 : 1);
}

// Node index on the grid: periodic wrap (valid for i in [-n, 2n)) or, on an
// extrapolating axis, the nearest boundary node.  Branch-free.
__device__ __forceinline__ int wrap_idx(int i, int n, int bc) {
  int w = i + ((i < 0) ? n : 0);
  w -= (w >= n) ? n : 0;
  const int c = min(max(i, 0), n - 1);
  return bc ? c : w;
}

// ---------------------------------------------------------------------------
// Interpolation of one population of A arrays into registers
// ---------------------------------------------------------------------------

template <int SET, int NS, int A, int ST, int RO>
struct Tile {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  static constexpr int D = S::D;
  static constexpr int TX = 64;
  // waves per block: eight (a 64x8xRO tile, less y halo per cell) where two
  // such blocks still fit on a compute unit and measured faster: the 17-21
  // velocity sets (3 %); four elsewhere (the D3Q45 f + g kernels: 64x8x2
  // measured 9 % slower than 64x4x2 in FP32, 14-15 % in 16-bit)
  // (cell-wise support: four, a whole number of cells)
  static constexpr int NW =
      (!Support<NS>::glc && D == 3 && A == 1 && RO == 4 && S::Q > 16 && S::Q <= 21) ? 8 : 4;
  static constexpr int NT = 64 * NW;                 // threads per block
  static constexpr int H = Support<NS>::halo;
  static constexpr int PX = TX + ((H + 2) & ~1);     // widest LDS row (even: pairs of x)
  static constexpr int PM = (D == 3) ? NW + H : NW;  // rows per outer plane in P
  static constexpr int TOUT = (D == 3) ? RO : NW * RO;  // outer extent of the tile
  static constexpr int PSZ = A * RO * PM * PX;       // one P buffer
  static constexpr int TSZ = (D == 3) ? A * RO * NW * PX : 1;
};

// Per-thread / per-block geometry
struct Geo {
  const void* glcx;      // cell-wise support: compact table [Q][3][p][8] (global)
  const void* xlds;      // cell-wise support: the x entries [Q][p][8], staged in LDS
  int x0, m0, o0;        // tile origin: inner (x), middle (y, 3D), outer (z or y)
  int nx, nm, no;        // extents along inner, middle, outer
  int bcx, bcm, bco;
  int sm, so;            // element strides of middle and outer axes
  int vx, vm, vo;        // valid extents of the tile along each axis
  int lane, w, tid;
};

// The stencil tables are read-only for the whole launch: reading them through
// the constant address space lets the compiler use scalar loads (one fetch
// per wave, no vector-memory round trip before the data loads).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
  return (cptr<T>)(p);
}

// Element at a 32-bit element offset from a per-population base pointer
// (the host guarantees that one population spans less than 4 GiB), so that
// loads use a scalar base and a 32-bit vector offset.
template <typename E>
__device__ __forceinline__ const E* at(const E* base, int e) {
  return reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + uint32_t(e) * uint32_t(sizeof(E)));
}
template <typename E>
__device__ __forceinline__ E* at(E* base, int e) {
  return reinterpret_cast<E*>(reinterpret_cast<char*>(base) + uint32_t(e) * uint32_t(sizeof(E)));
}

// First population whose velocity component along `axis` equals q's.  The
// stencil offset and weights along an axis depend on that component only, so
// indexing the tables by this representative lets the compiler share the
// offsets, weights and column addresses between populations.
template <int SET, int axis>
constexpr int axis_rep(int q) {
  using S = Set<SET>;
  for (int k = 0; k < q; ++k)
    if (S::xh(k, axis) == S::xh(q, axis)) return k;
  return q;
}

// Shape of population q's work: which axes move (and so need n taps and a
// halo), how many source columns stage A covers, and in how many rounds of
// the block's threads.
template <int SET, int NS, int A, int ST, int RO, int q>
struct PopShape {
  using TL = Tile<SET, NS, A, ST, RO>;
  using S = typename TL::S;
  static constexpr int D = S::D;
  static constexpr bool mx = NS > 1 && S::moves(q, 0);
  static constexpr bool mm = NS > 1 && D == 3 && S::moves(q, 1);
  static constexpr bool mo = NS > 1 && S::moves(q, D - 1);
  static constexpr bool direct = !mx && !mm;  // no LDS: each thread loads its own column
  using SP = Support<NS>;
  // cell-wise support: along x and y the tile is a whole number of cells and
  // needs p + 1 more source nodes; along the outer axis a thread's RO rows lie
  // in one cell (RO divides p), whose window of 2p + 1 rows it loads
  static constexpr int HX = mx ? SP::halo : 0, HM = mm ? SP::halo : 0;
  static constexpr int HO = mo ? (SP::glc ? SP::win - RO : NS - 1) : 0;
  // taps: uniform NS per axis; cell-wise: the phase's own p + 1 along x and
  // y (from a per-phase first node), the padded window along the outer axis
  static constexpr int KX = mx ? (SP::glc ? SP::p + 1 : NS) : 1;
  static constexpr int KM = mm ? (SP::glc ? SP::p + 1 : NS) : 1;
  static constexpr int KO = mo ? SP::win : 1;
  static_assert(!SP::glc || (SP::p % RO == 0 && (D == 2 || TL::NW % SP::p == 0) && TL::TX % SP::p == 0),
                "cell-wise tiles must consist of whole cells");
  // 2D: a thread's outer rows are one cell, so that every load column's rows
  // have the phases 0..p-1 of the weights the thread holds
  static_assert(!SP::glc || D == 3 || RO == SP::p, "2D cell-wise tiles: one cell per thread");
  // 3D populations through LDS load x in pairs of adjacent nodes (one
  // two-element load per pair; the window starts at an even node, so it may
  // begin one node early: sh below)
  static constexpr bool X2 = D == 3 && !direct;
  static constexpr int CXL = TL::TX + HX;  // x columns the y and x passes use
  static constexpr int CX = X2 ? (mx ? (TL::TX + HX + 2) / 2 : TL::TX / 2) : CXL;  // load columns (pairs if X2)
  static constexpr int XW = X2 ? 2 : 1;   // x nodes per load column
  static constexpr int CM = (D == 3) ? TL::NW + HM : TL::NW;
  static constexpr int NCOL = CX * CM;
  static constexpr int ROUNDS = direct ? 1 : (NCOL + TL::NT - 1) / TL::NT;
  static_assert(!X2 || 2 * CX <= TL::PX, "LDS row too short for the pair window");
};

// Whether lanes past the last column of a partial round skip it with a branch
// rather than repeating the last column.  The branch costs the software
// pipeline (see pop_load), repeating costs the round's loads and stage A work.
// 2D tiles (68 load columns per 64-lane row at n = 5: a last round 6 % full)
// measured 13-17 % faster with the branch in FP64 storage and equal or 4-6 %
// slower in FP32; 3D rounds are full or nearly so.
template <int D, int ST>
constexpr bool skip_round_tail() {
  return D == 2 && ST == ST_F64;
}

// Everything population q needs after its loads were issued: the loaded
// values (still in flight until first use) and where each round's column
// lands in LDS.
template <int SET, int NS, int A, int ST, int RO, int q>
struct PopIn {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using R = typename StoreT<ST>::real;
  R v[PS::ROUNDS][A][RO + PS::HO][PS::XW];
  int slot[PS::ROUNDS];
  int sh;  // X2: the window starts sh (0 or 1) nodes before the stencil's first node
};

// Issue the HBM loads of population q (all A arrays) of `src` with stencil
// (off, wts).  With SUB every loaded value has ref[a] subtracted (exact for
// values within a factor two of the reference), so the interpolation works
// on deviations.
//
// XP (3D populations through LDS): 1 loads each pair of x nodes with one
// two-element load, valid when the launch has x periodic, nx even and
// buffers aligned to two elements (then a pair never straddles the wrap or a
// row end); 0 loads the two nodes singly (clamped x, odd nx, unaligned
// buffers).  Either way every lane issues the same loads with no branch:
// lanes past the last column repeat it (2D FP64 aside, skip_round_tail).  A
// branch around the loads (per lane or per launch) makes the compiler wait
// for every load in flight, the next population's included, before the first
// use of any of them, which undoes the software pipeline (Pipe).
template <int SET, int NS, int A, int ST, int RO, int q, bool SUB, int XP>
__device__ __forceinline__ void pop_load(const Geo& g, const typename StoreT<ST>::elem* __restrict__ src,
                                         int64_t pstride, const int* __restrict__ off,
                                         const typename StoreT<ST>::real* __restrict__ wts,
                                         const typename StoreT<ST>::real (&ref)[A],
                                         PopIn<SET, NS, A, ST, RO, q>& in) {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using TL = typename PS::TL;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  constexpr int D = PS::D;
  constexpr int Q = TL::S::Q;
  constexpr int HX = PS::HX, HM = PS::HM, HO = PS::HO;
  constexpr int axm = 1, axo = D - 1;

  // offsets through the axis representatives: populations with the same
  // component share their per-lane column addresses and scalar row offsets
  constexpr int qx = axis_rep<SET, 0>(q), qm = axis_rep<SET, axm>(q), qo = axis_rep<SET, axo>(q);
  const cptr<int> offc = as_const(off);
  const int ox = offc[3 * qx + 0];
  const int om = (D == 3) ? offc[3 * qm + axm] : 0;
  const int oo = offc[3 * qo + axo];

  const E* base[A];
#pragma unroll
  for (int a = 0; a < A; ++a) base[a] = src + int64_t(a * Q + q) * pstride;

  // element offset of load row r of a thread whose first cell row is ob (vob
  // valid rows): rows ob + oo .. (uniform stencil, dead rows repeat the last
  // valid one), or the window of the cell holding ob (cell-wise support)
  auto row_at = [&](int ob, int vob, int r) -> int {
    if constexpr (PS::SP::glc && PS::mo)
      return wrap_idx(ob - ob % PS::SP::p + oo + r, g.no, g.bco) * g.so;
    else
      return wrap_idx(ob + oo + min(r, vob - 1 + HO), g.no, g.bco) * g.so;
  };

  int col[PS::ROUNDS], ob[PS::ROUNDS], vo[PS::ROUNDS];
  int col2[PS::ROUNDS];  // X2 with single loads: column of the pair's second node
  in.sh = 0;
  if constexpr (PS::direct) {
    // each thread loads its own column
    col[0] = wrap_idx(g.x0 + min(g.lane, g.vx - 1) + ox, g.nx, g.bcx);
    ob[0] = g.o0;
    vo[0] = g.vo;
    if constexpr (D == 3) {
      col[0] += wrap_idx(g.m0 + min(g.w, g.vm - 1) + om, g.nm, g.bcm) * g.sm;
    } else {
      ob[0] = g.o0 + min(g.w * RO, g.vo - 1);  // a dead segment reads in-bounds rows
      vo[0] = max(1, min(RO, g.vo - g.w * RO));
    }
    in.slot[0] = 0;
  } else if constexpr (PS::X2) {
    // pairs (xa + 2j, xa + 2j + 1) from the even node xa at or below x0 + ox
    const int xs0 = g.x0 + ox;
    const int xa = g.x0 + (ox & ~1);
    in.sh = ox & 1;
    // one node beyond the last one the stencil needs: the nodes of the
    // columns past it (a partial tile) are never read
    const int xlim = xs0 + g.vx + HX;
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr) {
      const int c = min(g.tid + TL::NT * rr, PS::NCOL - 1);
      const int j = c % PS::CX, ms = c / PS::CX;
      in.slot[rr] = ms * TL::PX + 2 * j;
      const int e0 = max(min(xa + 2 * j, xlim), -g.nx), e1 = max(min(xa + 2 * j + 1, xlim), -g.nx);
      const int cm = wrap_idx(g.m0 + om + min(ms, g.vm - 1 + HM), g.nm, g.bcm) * g.sm;
      if constexpr (XP) {
        // periodic x, nx even: xa + 2j wraps to an even node whose successor
        // is the pair's second node; a start clamped at xlim (unread) is
        // rounded down to its pair
        col[rr] = (wrap_idx(min(e0, 2 * g.nx - 1), g.nx, 0) & ~1) + cm;
        col2[rr] = col[rr] + 1;
      } else {
        col[rr] = wrap_idx(min(e0, 2 * g.nx - 1), g.nx, g.bcx) + cm;
        col2[rr] = wrap_idx(min(e1, 2 * g.nx - 1), g.nx, g.bcx) + cm;
      }
    }
  } else {
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr) {
      const int c = min(g.tid + TL::NT * rr, PS::NCOL - 1);
      const int xs = c % PS::CX, ms = c / PS::CX;
      in.slot[rr] = ms * TL::PX + xs;
      col[rr] = wrap_idx(g.x0 + ox + min(xs, g.vx - 1 + HX), g.nx, g.bcx);
      if constexpr (D == 3) {
        col[rr] += wrap_idx(g.m0 + om + min(ms, g.vm - 1 + HM), g.nm, g.bcm) * g.sm;
        ob[rr] = g.o0;
        vo[rr] = g.vo;
      } else {
        ob[rr] = g.o0 + min(ms * RO, g.vo - 1);  // a dead segment reads in-bounds rows
        vo[rr] = max(1, min(RO, g.vo - ms * RO));
      }
    }
  }
  // 3D: the row is the same for the whole block, so its byte offset goes into
  // a scalar register and only the column offset is per lane
  rsrc_t rs[A];
  if constexpr (D == 3) {
#pragma unroll
    for (int a = 0; a < A; ++a) rs[a] = make_rsrc(base[a], pstride);
  }
  if constexpr (PS::X2) {
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr)
#pragma unroll
      for (int r = 0; r < RO + HO; ++r) {
        const int row = row_at(g.o0, g.vo, r);
#pragma unroll
        for (int a = 0; a < A; ++a) {
          if constexpr (XP) {
            TR::ldb2(rs[a], boff<E>(col[rr]), boff<E>(row), in.v[rr][a][r][0], in.v[rr][a][r][1]);
          } else {
            in.v[rr][a][r][0] = TR::ldb(rs[a], boff<E>(col[rr]), boff<E>(row));
            in.v[rr][a][r][1] = TR::ldb(rs[a], boff<E>(col2[rr]), boff<E>(row));
          }
        }
      }
  } else {
    constexpr bool SKIP = skip_round_tail<D, ST>() && !PS::direct && PS::NCOL % TL::NT != 0;
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr)
      if (!SKIP || rr + 1 < PS::ROUNDS || g.tid + TL::NT * rr < PS::NCOL)
#pragma unroll
      for (int r = 0; r < RO + HO; ++r) {
        const int row = row_at(ob[rr], vo[rr], r);
#pragma unroll
        for (int a = 0; a < A; ++a) {
          if constexpr (D == 3)
            in.v[rr][a][r][0] = TR::ldb(rs[a], boff<E>(col[rr]), boff<E>(row));
          else
            in.v[rr][a][r][0] = TR::ld(at(base[a], row + col[rr]));
        }
      }
  }
  if constexpr (SUB) {
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr)
#pragma unroll
      for (int a = 0; a < A; ++a)
#pragma unroll
        for (int r = 0; r < RO + HO; ++r)
#pragma unroll
          for (int k = 0; k < PS::XW; ++k) in.v[rr][a][r][k] -= ref[a];
  }
}

// Stencil weights of population q along x, y and the outer axis (scalar
// loads, read when the population is interpolated rather than with its HBM
// loads, so that they do not hold scalar registers while the loads are in
// flight).  Uniform support: one set per axis (wm[0], wo[0]).  Cell-wise
// support: along x the lane's own phase (first window node bx and p + 1
// weights, from the LDS copy of the compact table); along y one compact
// entry per phase of the tile's rows (bm, wm); along the outer axis the
// padded window weights of each of the thread's RO rows (wo[r]).
template <int SET, int NS, int A, int ST, int RO, int q>
struct PopW {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using R = typename StoreT<ST>::real;
  static constexpr bool G = PS::SP::glc;
  static constexpr int P = PS::SP::p;
  R wx[PS::KX], wm[G ? P : 1][PS::KM], wo[G ? RO : 1][PS::KO];
  int bx, bm[G ? P : 1];
  __device__ __forceinline__ PopW(const R* __restrict__ wts, const Geo& g) {
    constexpr int axm = 1, axo = PS::D - 1;
    const cptr<R> wc = as_const(wts);
    bx = 0;
    bm[0] = 0;
    if constexpr (!G) {
      // the weights along an axis depend on the velocity component only: read
      // them at the axis representative, so that populations share the loads
      constexpr int qx = axis_rep<SET, 0>(q), qm = axis_rep<SET, axm>(q), qo = axis_rep<SET, axo>(q);
#pragma unroll
      for (int k = 0; k < PS::KX; ++k) wx[k] = PS::mx ? wc[(3 * qx + 0) * NS + k] : R(1);
#pragma unroll
      for (int k = 0; k < PS::KM; ++k) wm[0][k] = PS::mm ? wc[(3 * qm + axm) * NS + k] : R(1);
#pragma unroll
      for (int k = 0; k < PS::KO; ++k) wo[0][k] = PS::mo ? wc[(3 * qo + axo) * NS + k] : R(1);
    } else {
      constexpr int XE = PS::SP::xent, W = PS::SP::win;
      if constexpr (PS::mx) {
        const R* e = static_cast<const R*>(g.xlds) + (q * P + g.lane % P) * XE;
        bx = int(e[0]);
#pragma unroll
        for (int t = 0; t < PS::KX; ++t) wx[t] = e[1 + t];
      } else {
        wx[0] = R(1);
      }
      if constexpr (PS::mm) {
        const cptr<R> gc = as_const(static_cast<const R*>(g.glcx));
#pragma unroll
        for (int k = 0; k < P; ++k) {
          bm[k] = int(gc[((3 * q + axm) * P + k) * XE]);
#pragma unroll
          for (int t = 0; t < PS::KM; ++t) wm[k][t] = gc[((3 * q + axm) * P + k) * XE + 1 + t];
        }
      } else {
#pragma unroll
        for (int k = 0; k < P; ++k) wm[k][0] = R(1);
      }
      // phase of the thread's first outer row; its RO rows lie in one cell
      const int ob = (PS::D == 3) ? g.o0 : g.o0 + g.w * RO;
      const int k0 = ob % P;
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        if constexpr (PS::mo) {
#pragma unroll
          for (int u = 0; u < W; ++u) wo[r][u] = wc[((3 * q + axo) * P + k0 + r) * W + u];
        } else {
          wo[r][0] = R(1);
        }
      }
    }
  }
};

// The interpolation of a loaded population runs in three stages:
//   A  outer-axis interpolation in registers; the result goes to LDS buffer P
//      (populations moving along x or y) or straight to out (the others);
//   B  y interpolation P -> T in LDS (populations moving along y, 3D);
//   C  x interpolation from P or T into out.
// A block barrier separates A from B and B from C.
template <int SET, int NS, int A, int ST, int RO, int q>
__device__ __forceinline__ void stage_A(const Geo& g, PopIn<SET, NS, A, ST, RO, q>& in,
                                        const PopW<SET, NS, A, ST, RO, q>& w, typename StoreT<ST>::real* P,
                                        typename StoreT<ST>::real (&out)[A][RO]) {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using TL = typename PS::TL;
  using R = typename StoreT<ST>::real;
  constexpr int KO = PS::KO;
  constexpr int PX = TL::PX, PM = TL::PM;
  constexpr int XW = PS::XW;
  // outer-axis interpolation of x node k of one load column
  auto outer = [&](const R (&v)[A][RO + PS::HO][XW], int k, R (&res)[A][RO]) {
#pragma unroll
    for (int a = 0; a < A; ++a)
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        if constexpr (KO == 1) {
          res[a][r] = v[a][r][k];
        } else if constexpr (PS::SP::glc) {
          // the padded window of the row's cell, weights of the row's phase
          R s = v[a][0][k] * w.wo[r][0];
#pragma unroll
          for (int u = 1; u < KO; ++u) s = fma(w.wo[r][u], v[a][u][k], s);
          res[a][r] = s;
        } else {
          R s = v[a][r][k] * w.wo[0][0];
#pragma unroll
          for (int t = 1; t < KO; ++t) s = fma(w.wo[0][t], v[a][r + t][k], s);
          res[a][r] = s;
        }
      }
  };
  if constexpr (PS::direct) {
    outer(in.v[0], 0, out);
  } else {
    // lanes past the last column repeat it (the same value to the same slot)
    // or skip it (skip_round_tail)
    constexpr bool SKIP = skip_round_tail<PS::D, ST>() && PS::NCOL % TL::NT != 0;
#pragma unroll
    for (int rr = 0; rr < PS::ROUNDS; ++rr)
      if (!SKIP || rr + 1 < PS::ROUNDS || g.tid + TL::NT * rr < PS::NCOL)
#pragma unroll
      for (int k = 0; k < XW; ++k) {
        R res[A][RO];
        outer(in.v[rr], k, res);
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
          for (int r = 0; r < RO; ++r) P[(a * RO + r) * PM * PX + in.slot[rr] + k] = res[a][r];
      }
  }
}

// y interpolation in LDS, one thread per (a, r, x) column
template <int SET, int NS, int A, int ST, int RO, int q>
__device__ __forceinline__ void stage_B(const Geo& g, const PopW<SET, NS, A, ST, RO, q>& w, int sh,
                                        const typename StoreT<ST>::real* P, typename StoreT<ST>::real* T) {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using TL = typename PS::TL;
  using R = typename StoreT<ST>::real;
  constexpr int KM = PS::KM, HM = PS::HM;
  constexpr int PX = TL::PX, PM = TL::PM;
  if constexpr (PS::mm) {
    constexpr int NB = A * RO * PS::CXL;
#pragma unroll
    for (int c0 = 0; c0 < NB; c0 += TL::NT) {
      const int c = c0 + g.tid;
      if (NB % TL::NT == 0 || c < NB) {
        const int xs = c % PS::CXL, ar = c / PS::CXL;
        if constexpr (PS::SP::glc) {
          // row m (phase m % p): p + 1 rows from its cell's first window row
          constexpr int PP = PS::SP::p;
#pragma unroll
          for (int m = 0; m < TL::NW; ++m) {
            const R* col = P + (ar * PM + (m - m % PP) + w.bm[m % PP]) * PX + xs + sh;
            R s = col[0] * w.wm[m % PP][0];
#pragma unroll
            for (int k = 1; k < KM; ++k) s = fma(w.wm[m % PP][k], col[k * PX], s);
            T[(ar * TL::NW + m) * PX + xs] = s;
          }
        } else {
          R colv[TL::NW + HM];
#pragma unroll
          for (int m = 0; m < TL::NW + HM; ++m) colv[m] = P[(ar * PM + m) * PX + xs + sh];
#pragma unroll
          for (int m = 0; m < TL::NW; ++m) {
            R s = colv[m] * w.wm[0][0];
#pragma unroll
            for (int k = 1; k < KM; ++k) s = fma(w.wm[0][k], colv[m + k], s);
            T[(ar * TL::NW + m) * PX + xs] = s;
          }
        }
      }
    }
  }
}

// x interpolation from LDS into registers (populations that use LDS)
template <int SET, int NS, int A, int ST, int RO, int q>
__device__ __forceinline__ void stage_C(const Geo& g, const PopW<SET, NS, A, ST, RO, q>& w, int sh,
                                        const typename StoreT<ST>::real* P, const typename StoreT<ST>::real* T,
                                        typename StoreT<ST>::real (&out)[A][RO]) {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  using TL = typename PS::TL;
  using R = typename StoreT<ST>::real;
  constexpr int KX = PS::KX;
  constexpr int PX = TL::PX, PM = TL::PM;
  if constexpr (!PS::direct) {
    const R* X = PS::mm ? T : P;              // rows [a][r][row][x], row = wave
    constexpr int XR = PS::mm ? TL::NW : PM;  // rows per (a, r) plane of X
#pragma unroll
    for (int a = 0; a < A; ++a)
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        // cell-wise support: the lane's cell's first window node, plus its phase's offset
        const int lx = PS::SP::glc && PS::mx ? g.lane - g.lane % PS::SP::p + w.bx : g.lane;
        const R* row = X + ((a * RO + r) * XR + g.w) * PX + lx + (PS::mm ? 0 : sh);
        if constexpr (KX == 1) {
          out[a][r] = row[0];
        } else {
          R s = row[0] * w.wx[0];
#pragma unroll
          for (int k = 1; k < KX; ++k) s = fma(w.wx[k], row[k], s);
          out[a][r] = s;
        }
      }
  }
}

// Finish the interpolation where it is written: without this the compiler
// sinks the last pass to the collision and keeps every population's raw taps
// alive.
template <int A, int RO, typename R>
__device__ __forceinline__ void pin(R (&out)[A][RO]) {
#pragma unroll
  for (int a = 0; a < A; ++a)
#pragma unroll
    for (int r = 0; r < RO; ++r) asm volatile("" : "+v"(out[a][r]));
}

// Interpolate the loaded population q into out[a][r] using LDS buffers P, T.
template <int SET, int NS, int A, int ST, int RO, int q>
__device__ __forceinline__ void pop_finish(const Geo& g, PopIn<SET, NS, A, ST, RO, q>& in,
                                           const typename StoreT<ST>::real* __restrict__ wts,
                                           typename StoreT<ST>::real* P, typename StoreT<ST>::real* T,
                                           typename StoreT<ST>::real (&out)[A][RO]) {
  using PS = PopShape<SET, NS, A, ST, RO, q>;
  const PopW<SET, NS, A, ST, RO, q> w(wts, g);
  stage_A(g, in, w, P, out);
  if constexpr (!PS::direct) {
    __syncthreads();
    if constexpr (PS::mm) {
      stage_B(g, w, in.sh, P, T);
      __syncthreads();
    }
    stage_C(g, w, in.sh, P, T, out);
  }
  pin(out);
}

// Two populations through the same barriers: twice the independent work
// between block synchronizations and half the synchronizations.
template <int SET, int NS, int A, int ST, int RO, int q0, int q1>
__device__ __forceinline__ void pair_finish(const Geo& g, PopIn<SET, NS, A, ST, RO, q0>& in0,
                                            PopIn<SET, NS, A, ST, RO, q1>& in1,
                                            const typename StoreT<ST>::real* __restrict__ wts,
                                            typename StoreT<ST>::real* P0, typename StoreT<ST>::real* P1,
                                            typename StoreT<ST>::real* T0, typename StoreT<ST>::real* T1,
                                            typename StoreT<ST>::real (&out0)[A][RO],
                                            typename StoreT<ST>::real (&out1)[A][RO]) {
  using PS0 = PopShape<SET, NS, A, ST, RO, q0>;
  using PS1 = PopShape<SET, NS, A, ST, RO, q1>;
  const PopW<SET, NS, A, ST, RO, q0> w0(wts, g);
  const PopW<SET, NS, A, ST, RO, q1> w1(wts, g);
  stage_A(g, in0, w0, P0, out0);
  stage_A(g, in1, w1, P1, out1);
  if constexpr (!PS0::direct || !PS1::direct) {
    __syncthreads();
    if constexpr (PS0::mm || PS1::mm) {
      stage_B(g, w0, in0.sh, P0, T0);
      stage_B(g, w1, in1.sh, P1, T1);
      __syncthreads();
    }
    stage_C(g, w0, in0.sh, P0, T0, out0);
    stage_C(g, w1, in1.sh, P1, T1, out1);
  }
  pin(out0);
  pin(out1);
}

// Whether population q uses LDS (needs the block-wide passes).
template <int SET, int NS, int q>
constexpr bool uses_lds() {
  using S = Set<SET>;
  return NS > 1 && (S::moves(q, 0) || (S::D == 3 && S::moves(q, 1)));
}

template <int SET, int NS, int q>
constexpr int lds_rank() {  // number of LDS-using populations before q
  int c = 0;
  if constexpr (q > 0) c = lds_rank<SET, NS, q - 1>() + (uses_lds<SET, NS, q - 1>() ? 1 : 0);
  return c;
}

// Software pipeline over the populations.  GROUP 1: the HBM loads of
// population q + 1 are issued before population q is interpolated, so their
// latency overlaps with q's LDS passes and barriers.  GROUP 2: the rest
// population first, then the others in pairs that share their barriers; the
// loads of the next pair are issued before a pair is interpolated.  LDS: Pb holds NPBUF buffers of Tile::PSZ, Tb two of
// Tile::TSZ; consecutive users of LDS alternate between buffers so that a
// population's stage A never overwrites what a lagging wave still reads.
// `sink(q, out)` receives each result.
template <int SET, int NS, int A, int ST, int RO, bool SUB, int PARITY, int GROUP, int XP>
struct Pipe {
  using R = typename StoreT<ST>::real;
  using E = typename StoreT<ST>::elem;
  using TL = Tile<SET, NS, A, ST, RO>;
  static constexpr int Q = Set<SET>::Q;
  static constexpr int NPBUF = 2 * GROUP;

  static __device__ __forceinline__ void refs(int q, R cv2, R (&ref)[A]) {
    ref[0] = SUB ? R(Set<SET>::T.w[q]) : R(0);
    if constexpr (A == 2) ref[1] = SUB ? cv2 * R(Set<SET>::T.w[q]) : R(0);
  }

  template <int q>
  static __device__ __forceinline__ void load(const Geo& g, const E* __restrict__ src, int64_t pstride,
                                              const int* __restrict__ off, const R* __restrict__ wts, R cv2,
                                              PopIn<SET, NS, A, ST, RO, q>& in) {
    R ref[A];
    refs(q, cv2, ref);
    pop_load<SET, NS, A, ST, RO, q, SUB, XP>(g, src, pstride, off, wts, ref, in);
  }

  template <int q, class Sink>
  static __device__ __forceinline__ void finish(const Geo& g, const R* __restrict__ wts, R* Pb, R* Tb,
                                                PopIn<SET, NS, A, ST, RO, q>& cur, Sink&& sink) {
    constexpr int buf = (lds_rank<SET, NS, q>() + PARITY) & 1;
    R o[A][RO];
    pop_finish<SET, NS, A, ST, RO, q>(g, cur, wts, Pb + buf * TL::PSZ, Tb + buf * TL::TSZ, o);
    sink(std::integral_constant<int, q>{}, o);
  }

  // one population in flight ahead: cur (q) is loaded on entry
  template <int q, class Sink>
  static __device__ __forceinline__ void run(const Geo& g, const E* __restrict__ src, int64_t pstride,
                                             const int* __restrict__ off, const R* __restrict__ wts, R cv2,
                                             R* Pb, R* Tb, PopIn<SET, NS, A, ST, RO, q>& cur, Sink&& sink) {
    if constexpr (q + 1 < Q) {
      PopIn<SET, NS, A, ST, RO, q + 1> nxt;
      load<q + 1>(g, src, pstride, off, wts, cv2, nxt);
      finish<q>(g, wts, Pb, Tb, cur, sink);
      run<q + 1>(g, src, pstride, off, wts, cv2, Pb, Tb, nxt, sink);
    } else {
      finish<q>(g, wts, Pb, Tb, cur, sink);
    }
  }

  // pairs: c0 (q) and c1 (q + 1) are loaded on entry; pair k = (q - 1) / 2
  template <int q, class Sink>
  static __device__ __forceinline__ void run_pairs(const Geo& g, const E* __restrict__ src, int64_t pstride,
                                                   const int* __restrict__ off, const R* __restrict__ wts, R cv2,
                                                   R* Pb, R* Tb, PopIn<SET, NS, A, ST, RO, q>& c0,
                                                   PopIn<SET, NS, A, ST, RO, q + 1>& c1, Sink&& sink) {
    constexpr int slot = ((((q - 1) / 2) + PARITY) & 1) * 2;
    R o0[A][RO], o1[A][RO];
    auto fin = [&]() {
      pair_finish<SET, NS, A, ST, RO, q, q + 1>(g, c0, c1, wts, Pb + slot * TL::PSZ, Pb + (slot + 1) * TL::PSZ,
                                                Tb, Tb + TL::TSZ, o0, o1);
      sink(std::integral_constant<int, q>{}, o0);
      sink(std::integral_constant<int, q + 1>{}, o1);
    };
    if constexpr (q + 3 < Q) {
      PopIn<SET, NS, A, ST, RO, q + 2> n0;
      PopIn<SET, NS, A, ST, RO, q + 3> n1;
      load<q + 2>(g, src, pstride, off, wts, cv2, n0);
      load<q + 3>(g, src, pstride, off, wts, cv2, n1);
      fin();
      run_pairs<q + 2>(g, src, pstride, off, wts, cv2, Pb, Tb, n0, n1, sink);
    } else {
      fin();
    }
  }

  template <class Sink>
  static __device__ __forceinline__ void all(const Geo& g, const E* __restrict__ src, int64_t pstride,
                                             const int* __restrict__ off, const R* __restrict__ wts, R cv2,
                                             R* Pb, R* Tb, Sink&& sink) {
    PopIn<SET, NS, A, ST, RO, 0> first;
    load<0>(g, src, pstride, off, wts, cv2, first);
    if constexpr (GROUP == 2) {
      static_assert(Q % 2 == 1 && !uses_lds<SET, NS, 0>(), "pairs need the rest population first");
      PopIn<SET, NS, A, ST, RO, 1> p1;
      PopIn<SET, NS, A, ST, RO, 2> p2;
      load<1>(g, src, pstride, off, wts, cv2, p1);
      load<2>(g, src, pstride, off, wts, cv2, p2);
      finish<0>(g, wts, Pb, Tb, first, sink);
      run_pairs<1>(g, src, pstride, off, wts, cv2, Pb, Tb, p1, p2, sink);
    } else {
      run<0>(g, src, pstride, off, wts, cv2, Pb, Tb, first, sink);
    }
  }

  // parity the next pipeline over the same LDS buffers must start with
  static constexpr int next_parity() {
    return GROUP == 2 ? (((Q - 1) / 2 + PARITY) & 1) : ((lds_rank<SET, NS, Q>() + PARITY) & 1);
  }
};

// Populations grouped per pair of barriers in the forward pass (one at a
// time for the cell-wise support, whose wider windows hold more registers).
template <int D, int NS, int A, int ST, int MODE>
constexpr int pipe_group() {
  return (D == 3 && A == 1 && is_step(MODE) && !Support<NS>::glc) ? 2 : 1;
}

// ---------------------------------------------------------------------------
// Equilibrium polynomial P(a, U, eta, X) = f^eq / (w rho), minus 1
// (App. A contracted with T0 = c_s^2; a = xh . u~, U = |u~|^2, X = |xh|^2,
// eta = theta - 1; the eta terms vanish in the weakly compressible model).
// ---------------------------------------------------------------------------

template <int N, int D, bool COMP, typename R>
__device__ __forceinline__ R peq_minus1(R a, R U, R eta, R X) {
  R a2 = a * a;
  R s = fma(a, fma(R(0.5), a, R(1)), R(-0.5) * U);  // a + (a^2 - U) / 2
  if constexpr (COMP) s += R(0.5) * eta * (X - R(D));
  if constexpr (N >= 3) {
    R t = a * (a2 - R(3) * U);
    if constexpr (COMP) t += R(3) * eta * a * (X - R(D + 2));
    s += t * R(1.0 / 6.0);
  }
  if constexpr (N >= 4) {
    R t = a2 * a2 - R(6) * a2 * U + R(3) * U * U;
    if constexpr (COMP) {
      t += R(6) * eta * ((X - R(D + 4)) * a2 - (X - R(D + 2)) * U);
      t += R(3) * eta * eta * (X * X - R(2 * (D + 2)) * X + R(D * (D + 2)));
    }
    s += t * R(1.0 / 24.0);
  }
  return s;
}

// Derivatives of P with respect to a and U (weakly compressible, eta = 0).
// sum_i w_i (P_i - 1) for the compressible N = 4 equilibrium with the rounded
// constants, from the moment defects c = KParams::mdef: the sum is linear in
// the set's moments and vanishes for the exact ones (Gaussian moments to
// degree 4), so it is the same polynomial evaluated on the defects alone.
template <int D, typename R>
__device__ __forceinline__ R peq_mass_defect(const double* c, R ux, R uy, R uz, R U, R eta) {
  const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
  const R W2 = R(c[1]) * x2 + R(c[2]) * y2 + R(c[3]) * z2 + R(c[4]) * ux * uy + R(c[5]) * ux * uz + R(c[6]) * uy * uz;
  const R WX2 = R(c[8]) * x2 + R(c[9]) * y2 + R(c[10]) * z2 + R(c[11]) * ux * uy + R(c[12]) * ux * uz +
                R(c[13]) * uy * uz;
  const R W4 = R(c[15]) * x2 * x2 + R(c[16]) * y2 * y2 + R(c[17]) * z2 * z2 + R(c[18]) * x2 * ux * uy +
               R(c[19]) * x2 * ux * uz + R(c[20]) * y2 * uy * ux + R(c[21]) * y2 * uy * uz + R(c[22]) * z2 * uz * ux +
               R(c[23]) * z2 * uz * uy + R(c[24]) * x2 * y2 + R(c[25]) * x2 * z2 + R(c[26]) * y2 * z2 +
               R(c[27]) * x2 * uy * uz + R(c[28]) * y2 * ux * uz + R(c[29]) * z2 * ux * uy;
  const R d0 = R(c[0]), dX = R(c[7]), dXX = R(c[14]);
  R S = R(0.5) * (W2 - U * d0) + R(0.5) * eta * (dX - R(D) * d0);
  const R t = W4 - R(6) * U * W2 + R(3) * U * U * d0 +
              R(6) * eta * (WX2 - R(D + 4) * W2 - (dX - R(D + 2) * d0) * U) +
              R(3) * eta * eta * (dXX - R(2 * (D + 2)) * dX + R(D * (D + 2)) * d0);
  return fma(t, R(1.0 / 24.0), S);
}

template <int N, typename R>
__device__ __forceinline__ void peq_derivs(R a, R U, R& P, R& Pa, R& PU) {
  R a2 = a * a;
  P = R(1) + a + R(0.5) * (a2 - U);
  Pa = R(1) + a;
  PU = R(-0.5);
  if constexpr (N >= 3) {
    P += a * (a2 - R(3) * U) * R(1.0 / 6.0);
    Pa += R(0.5) * (a2 - U);
    PU -= R(0.5) * a;
  }
  if constexpr (N >= 4) {
    P += (a2 * a2 - R(6) * a2 * U + R(3) * U * U) * R(1.0 / 24.0);
    Pa += a * (a2 - R(3) * U) * R(1.0 / 6.0);
    PU += R(0.25) * (U - a2);
  }
}

// ---------------------------------------------------------------------------
// The fused kernel
// ---------------------------------------------------------------------------

// Threads per block of the fused kernel.
template <int SET, int NS, int A, int ST, int MODE>
constexpr int sl_threads() {
  return Tile<SET, NS, A, ST, cells_per_thread<Set<SET>::D, Set<SET>::Q, A, ST, MODE>()>::NT;
}

// Minimum waves per SIMD the register allocation must allow: two for the
// FP32 quasi-equilibrium f + g step in 3D (two cells per thread; its heat
// fluxes would take it to 273 registers, one wave per SIMD: 17 spilled
// registers cost less, D3Q45 at 256^3 5.92 against 7.68 ms), else no bound.
template <int SET, int NS, int A, int ST, int MODE>
constexpr int sl_min_waves() {
  return (Set<SET>::D == 3 && A == 2 && ST == ST_F32 && MODE == MODE_STEP_QE) ? 2 : 1;
}

// CP: cache policy of the result stores (0 or CP_STREAM).  XP: x pairs
// loaded with one two-element load (1) or singly (0), see pop_load.  RND:
// 16-bit step stores round to nearest (0) or stochastically (1; a variant of
// its own, so that the default keeps its code size and schedule).
template <int SET, int NS, int N, int A, int ST, int MODE, int CP, int XP, int RND = 0>
__global__ __launch_bounds__((sl_threads<SET, NS, A, ST, MODE>()), (sl_min_waves<SET, NS, A, ST, MODE>()))
void sl_kernel(KParams p) {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  constexpr int D = S::D;
  constexpr int Q = S::Q;
  constexpr bool DEV = TR::dev;
  constexpr bool COMP = (A == 2);
  // the energy moment summed in FP64 (16-bit compressible storage only; the
  // host rejects it elsewhere, so other kernels carry none of its code)
  constexpr bool E64 = TR::coarse && COMP;
  constexpr int RO = cells_per_thread<D, Q, A, ST, MODE>();
  using TL = Tile<SET, NS, A, ST, RO>;

  constexpr int GROUP = pipe_group<D, NS, A, ST, MODE>();
  __shared__ __align__(16) R P_lds[2 * GROUP][TL::PSZ];
  __shared__ __align__(16) R T_lds[2][TL::TSZ];
  // cell-wise support: the compact x entries of every population and phase
  using SP = Support<NS>;
  constexpr int XT = SP::glc ? Q * SP::p * SP::xent : 1;
  __shared__ __align__(16) R X_lds[XT];

  Geo g;
  g.glcx = p.glcx;
  g.xlds = X_lds;
  g.tid = threadIdx.x;
  g.lane = threadIdx.x & 63;
  g.w = threadIdx.x >> 6;
  g.nx = p.n[0];
  g.bcx = p.bc[0];
  // XCD-aware tile order: hardware blocks go round-robin to the 8 XCDs.  Each
  // XCD gets one block of the grid (3D: a 4 x 2 or 2 x 4 split of the y and
  // z tiles, the host's choice, so that the halo planes two XCDs both read
  // are few).  The XCD walks it so
  // that the tiles it holds at once, which read each other's halo rows, are
  // neighbours: x, y, z when its xy plane of tiles is small against the
  // blocks it runs at once (the z neighbours then run together too); else in
  // bricks of by x bz (y, z) tiles, z fastest, the bricks walked x, y, z, so
  // that tiles one or two cells thick along z do not wait a whole plane of
  // tiles for the neighbours that re-read three of their four source planes
  // (which L2 and the Infinity Cache no longer hold by then).
  const int bid = blockIdx.x;
  const int xcd = bid & 7, lt = bid >> 3;
  int tix, tiy, tiz;
  if (p.rsy > 0) {
    int ly, lz;
    if (p.bz > 0) {
      const int nby = (p.rsy + p.by - 1) / p.by;
      const int per = p.by * p.bz;
      const int brick = lt / per, w = lt % per;
      tix = brick % p.tiles[0];
      const int bb = brick / p.tiles[0];
      ly = (bb % nby) * p.by + w / p.bz;
      lz = (bb / nby) * p.bz + w % p.bz;
      if (ly >= p.rsy) return;
    } else {
      tix = lt % p.tiles[0];
      const int rest = lt / p.tiles[0];
      ly = rest % p.rsy;
      lz = rest / p.rsy;
    }
    tiy = (xcd & ((1 << p.ysl) - 1)) * p.rsy + ly;
    tiz = (xcd >> p.ysl) * p.rsz + lz;
    if (lz >= p.rsz || tiy >= p.tiles[1] || tiz >= p.tiles[2]) return;
  } else {
    const int tile = xcd * p.chunk + lt;
    if (tile >= p.tiles[0] * p.tiles[1] * p.tiles[2]) return;
    tix = tile % p.tiles[0];
    tiy = (tile / p.tiles[0]) % p.tiles[1];
    tiz = tile / (p.tiles[0] * p.tiles[1]);
  }
  g.x0 = tix * TL::TX;
  g.vx = min(TL::TX, g.nx - g.x0);
  if constexpr (D == 3) {
    g.nm = p.n[1]; g.no = p.n[2];
    g.bcm = p.bc[1]; g.bco = p.bc[2];
    g.sm = p.n[0]; g.so = p.n[0] * p.n[1];
    g.m0 = tiy * TL::NW;
    g.o0 = tiz * RO;
    g.vm = min(TL::NW, g.nm - g.m0);
    g.vo = min(RO, g.no - g.o0);
  } else {
    g.nm = 1; g.no = p.n[1];
    g.bcm = 0; g.bco = p.bc[1];
    g.sm = 0; g.so = p.n[0];
    g.m0 = 0;
    g.o0 = tiy * TL::TOUT;
    g.vm = 1;
    g.vo = min(TL::TOUT, g.no - g.o0);
  }

  if constexpr (SP::glc) {
    // stage the x entries ([Q][p][8] of the [Q][3][p][8] table) in LDS
    const R* __restrict__ gx = static_cast<const R*>(p.glcx);
    constexpr int PE = SP::p * SP::xent;
    for (int i = g.tid; i < XT; i += TL::NT) X_lds[i] = gx[(3 * (i / PE)) * PE + i % PE];
    __syncthreads();
  }

  const E* __restrict__ src = static_cast<const E*>(p.src);
  const R* __restrict__ wts = static_cast<const R*>(p.wts);
  const R* __restrict__ wts_t = static_cast<const R*>(p.wts_t);

  // interpolated populations of this thread's RO cells
  R ft[A * Q][RO];
  // second interpolated / local input for the adjoint modes
  constexpr bool TWO = (MODE == MODE_ADJ_STEP || MODE == MODE_ADJ_COLLIDE);
  R lam[TWO ? Q : 1][RO];

  // populations stored whole but computed on as deviations
  constexpr bool SUBREF = DEV && !TR::stores_dev;
  const R cv2 = R(p.cv2mD);

  if constexpr (MODE != MODE_ADJ_STREAM) {
    Pipe<SET, NS, A, ST, RO, SUBREF, 0, GROUP, XP>::all(g, src, p.pstride, p.off, wts, cv2, &P_lds[0][0],
                                                            &T_lds[0][0], [&](auto qc, R (&o)[A][RO]) {
      constexpr int q = decltype(qc)::value;
#pragma unroll
      for (int a = 0; a < A; ++a)
#pragma unroll
        for (int r = 0; r < RO; ++r) ft[a * Q + q][r] = o[a][r];
    });
  }
  if constexpr (MODE == MODE_ADJ_STEP || MODE == MODE_ADJ_STREAM) {
    // S^T applied to src2 with the transposed stencil; src2 is of the compute type
    const E* __restrict__ src2 = static_cast<const E*>(p.src2);
    constexpr int parity =
        (MODE == MODE_ADJ_STREAM) ? 0 : Pipe<SET, NS, A, ST, RO, SUBREF, 0, GROUP, XP>::next_parity();
    static_assert(MODE == MODE_ADJ_STREAM || A == 1, "adjoint kernels are built for one array");
    Pipe<SET, NS, 1, ST, RO, false, parity, 1, XP>::all(g, src2, p.pstride, p.off_t, wts_t, cv2, &P_lds[0][0],
                                                  &T_lds[0][0], [&](auto qc, R (&o)[1][RO]) {
      constexpr int q = decltype(qc)::value;
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        if constexpr (MODE == MODE_ADJ_STREAM) ft[q][r] = o[0][r];
        else lam[q][r] = o[0][r];
      }
    });
  }

  // cell coordinates of this thread's RO cells
  const int xi = g.x0 + g.lane;
  int mi = 0, obase = g.o0, ovalid = g.vo;
  if constexpr (D == 3) {
    mi = g.m0 + g.w;
  } else {
    obase = g.o0 + g.w * RO;
    ovalid = min(RO, g.vo - g.w * RO);
  }
  const bool live = (g.lane < g.vx) && (D == 2 || g.w < g.vm) && ovalid > 0;
  if (!live) return;

  E* __restrict__ dst = static_cast<E*>(p.dst);
  const E* __restrict__ lam_in = static_cast<const E*>(p.src2);

  // 3D: the row (obase + r) is uniform, so its byte offset goes into a scalar
  // register and each lane adds its offset within the row.  Rows past the
  // domain (a partial z tile) get an offset beyond the buffer, where the
  // hardware drops the store.
  auto lc_of = [&](int r) -> int { return (D == 3) ? mi * g.nx + xi : (obase + r) * g.nx + xi; };
  auto rowb_of = [&](int r) -> int {
    // one population's byte size: at or beyond the buffer's end, and with the
    // lane offset (less than one plane) still below 2^32
    return (D == 3) ? (r < ovalid ? boff<E>((obase + r) * g.so) : boff<E>(int(p.pstride))) : 0;
  };
  auto put_at = [&](int k, int r, R v) {  // store array k (population, or Q + population) of cell r
    if constexpr (RND) {  // stochastic rounding, bits from (cell, array, seed)
      static_assert((ST == ST_BF16 || ST == ST_F16) && is_step(MODE), "stochastic rounding: 16-bit step kernels");
      const uint32_t cell = uint32_t((D == 3) ? (obase + r) * g.so + lc_of(r) : lc_of(r));
      const uint32_t rnd = hash32((cell * uint32_t(A * Q) + uint32_t(k)) ^ p.seed);
      if constexpr (D == 3)
        TR::template stb_sr<CP>(v, rnd, make_rsrc(dst + int64_t(k) * p.pstride, p.pstride), boff<E>(lc_of(r)),
                                rowb_of(r));
      else
        TR::st_sr(at(dst + int64_t(k) * p.pstride, lc_of(r)), v, rnd);
      return;
    }
    if constexpr (D == 3)
      TR::template stb<CP>(v, make_rsrc(dst + int64_t(k) * p.pstride, p.pstride), boff<E>(lc_of(r)), rowb_of(r));
    else
      TR::st(at(dst + int64_t(k) * p.pstride, lc_of(r)), v);
  };

  // ---- moments of cell r (Sec. 3): rho, j~ = sum xh f, u~, and for the
  // compressible model the energy sums, theta and the local relaxation rate
  struct Mom {
    R rho, dr, ux, uy, uz, U, theta, eta, omega, Epre;
    double Epre64;
    // MODE_STEP_QE: the co-moving non-equilibrium heat fluxes of f and g and
    // the rate they relax at
    R qf[3], qg[3], omq;
  };
  auto moments = [&](int r) -> Mom {
    // ---- moments (Sec. 3): rho, j~ = sum xh f (and energy sums)
    R rho, drho = R(0), jx = R(0), jy = R(0), jz = R(0);
    R Ef = R(0), G = R(0);
    double Ed = 0.0;
    // total energy sum(|xh|^2 f + g) before the collision, in the frame the
    // equilibrium is formed in (deviations, or whole values for FP64)
    R Epre = R(0);
    double Epre64 = 0.0;
    if constexpr (DEV) {
      // plain sums of the deviations; with 16-bit storage the energy moment
      // may be summed term by term in FP64 instead (p.e64), a choice taken
      // once per cell: tested per term, it is compiled into selects that
      // compute both sums
      R sr = R(0), se = R(0), sg = R(0);
      auto sums = [&](auto e64c) {
        constexpr bool E64 = decltype(e64c)::value;
        static_for<Q>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          const R d = ft[q][r];
          sr += d;
          if constexpr (S::moves(q, 0)) jx = fma(R(S::xh(q, 0)), d, jx);
          if constexpr (S::moves(q, 1)) jy = fma(R(S::xh(q, 1)), d, jy);
          if constexpr (D == 3 && S::moves(q, 2)) jz = fma(R(S::xh(q, 2)), d, jz);
          if constexpr (COMP) {
            constexpr double X = S::xh(q, 0) * S::xh(q, 0) + S::xh(q, 1) * S::xh(q, 1) + S::xh(q, 2) * S::xh(q, 2);
            if constexpr (X != 0.0) {
              if constexpr (E64) Ed = fma(X, double(d), Ed);
              else se = fma(R(X), d, se);
            }
            sg += ft[Q + q][r];
          }
        });
      };
      if constexpr (E64) {
        if (p.e64 != 0.0) sums(std::true_type{});
        else sums(std::false_type{});
      } else {
        sums(std::false_type{});
      }
      drho = R(p.sw - 1.0) + sr;
      rho = R(p.sw) + sr;
      jx += R(p.swx[0]);
      jy += R(p.swx[1]);
      jz += R(p.swx[2]);
      if constexpr (COMP) {
        // (se = 0 when Ed holds the FP64 sum, Ed = 0 otherwise)
        Ed += double(se);
        Epre64 = Ed + double(sg);
        Epre = se + sg;
        Ed += p.swX;
        Ef = R(p.swX) + se;
        G = R(p.cv2mD * p.sw) + sg;
      }
    } else {
      rho = R(0);
      static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const R f = ft[q][r];
        rho += f;
        if constexpr (S::moves(q, 0)) jx = fma(R(S::xh(q, 0)), f, jx);
        if constexpr (S::moves(q, 1)) jy = fma(R(S::xh(q, 1)), f, jy);
        if constexpr (D == 3 && S::moves(q, 2)) jz = fma(R(S::xh(q, 2)), f, jz);
        if constexpr (COMP) {
          constexpr double X = S::xh(q, 0) * S::xh(q, 0) + S::xh(q, 1) * S::xh(q, 1) + S::xh(q, 2) * S::xh(q, 2);
          if constexpr (X != 0.0) Ef = fma(R(X), f, Ef);
          G += ft[Q + q][r];
        }
      });
    }
    R ux, uy, uz;
    if constexpr (DEV) {
      // u~ = j~ + j~ (1/rho - 1) with 1/rho - 1 = -drho/rho: one rounding on
      // j~'s own bits.  Rounding 1/rho itself is biased for rho within a few
      // ulps of 1 (the reciprocal of a float just below 1 falls on or next to
      // a midpoint of the coarser grid above 1), a bias of ~1e-9 in u~ that BGK
      // with omega near 2 turns into a steady growth of the kinetic energy.
      const R im1 = -drho / rho;
      ux = fma(jx, im1, jx);
      uy = fma(jy, im1, jy);
      uz = (D == 3) ? fma(jz, im1, jz) : R(0);
    } else {
      const R inv_rho = R(1) / rho;
      ux = jx * inv_rho;
      uy = jy * inv_rho;
      uz = (D == 3) ? jz * inv_rho : R(0);
    }
    const R U = ux * ux + uy * uy + uz * uz;

    Mom m;
    m.rho = rho;
    m.dr = DEV ? drho : rho - R(1);
    m.ux = ux; m.uy = uy; m.uz = uz; m.U = U;
    m.Epre = Epre;
    m.Epre64 = Epre64;
    m.theta = R(1); m.eta = R(0); m.omega = R(p.omega);
    if constexpr (is_step(MODE)) {
      R omega = R(p.omega), theta = R(1), eta = R(0);
      if constexpr (COMP) {
        // 2 rho C_v theta = sum |xh - u~|^2 f + sum g = E_f - rho U + G
        if constexpr (DEV) {
          // in deviations: 2 C_v rho (theta - 1) = E~ - rho U - 2 C_v (rho - 1),
          // E~ = sum |xh|^2 (f - w) + sum (g - (2 C_v - D) w), so that theta - 1
          // is formed from small quantities (no cancellation against 2 C_v)
          const double twocv = 1.0 / p.inv2cv;
          const double e0 = p.swX + p.cv2mD * p.sw - twocv;  // zero up to rounding of the table sums
          if (E64 && p.e64 != 0.0) {
            const double et = (Epre64 + e0 - double(rho) * double(U) - twocv * double(drho)) * p.inv2cv / double(rho);
            eta = R(et);
            theta = R(1.0 + et);
          } else {
            eta = (Epre + R(e0) - rho * U - R(twocv) * drho) * R(p.inv2cv) / rho;
            theta = R(1) + eta;
          }
        } else {
          theta = (Ef - rho * U + G) * R(p.inv2cv) / rho;
          eta = theta - R(1);
        }
        // tau = 1/2 + (tau_ref - 1/2) / (rho theta)
        const R tau = R(0.5) + R(p.tau_m_half) / (rho * theta);
        omega = R(1) / tau;
      }
      m.theta = theta; m.eta = eta; m.omega = omega;
    }
    if constexpr (MODE == MODE_STEP_QE) {
      // Quasi-equilibrium (Pr != 1): heat fluxes in the frame moving with the
      // fluid, non-equilibrium parts, from the set's moments of the
      // interpolated populations minus the equilibrium's closed forms
      // (exact for sets of degree >= 7 at N = 4): contracted third moment
      // rho u~ (U + (D + 2) theta), stress rho (u~ u~ + theta I), g flux
      // (2 C_v - D) theta rho u~.  With deviation storage the sums run over
      // f - w and g - (2 C_v - D) w, whose references carry I and 2 C_v - D.
      R qa[3] = {R(0), R(0), R(0)}, ga[3] = {R(0), R(0), R(0)}, pa[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
      R ea = R(0), gs = R(0);
      static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr double x0 = S::xh(q, 0), x1 = S::xh(q, 1), x2 = S::xh(q, 2);
        constexpr double X = x0 * x0 + x1 * x1 + x2 * x2;
        const R d = ft[q][r], e = ft[Q + q][r];
        if constexpr (X != 0.0) ea = fma(R(X), d, ea);
        gs += e;
        if constexpr (x0 != 0.0) { qa[0] = fma(R(x0 * X), d, qa[0]); ga[0] = fma(R(x0), e, ga[0]); pa[0] = fma(R(x0 * x0), d, pa[0]); }
        if constexpr (x1 != 0.0) { qa[1] = fma(R(x1 * X), d, qa[1]); ga[1] = fma(R(x1), e, ga[1]); pa[1] = fma(R(x1 * x1), d, pa[1]); }
        if constexpr (x2 != 0.0) { qa[2] = fma(R(x2 * X), d, qa[2]); ga[2] = fma(R(x2), e, ga[2]); pa[2] = fma(R(x2 * x2), d, pa[2]); }
        if constexpr (x0 * x1 != 0.0) pa[3] = fma(R(x0 * x1), d, pa[3]);
        if constexpr (x0 * x2 != 0.0) pa[4] = fma(R(x0 * x2), d, pa[4]);
        if constexpr (x1 * x2 != 0.0) pa[5] = fma(R(x1 * x2), d, pa[5]);
      });
      const R rho_ = m.rho, th = m.theta;
      const R u[3] = {m.ux, m.uy, m.uz};
      // rho theta less the reference the sums exclude (deviations: 1)
      const R rt = DEV ? fma(rho_, m.eta, m.dr) : rho_ * th;
      const R cv2r = R(p.cv2mD);
      const R trp = ea - rho_ * m.U - R(D) * rt;
      R pn[3][3];
      const int pi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) pn[a][b] = pa[pi[a][b]] - rho_ * u[a] * u[b] - (a == b ? rt : R(0));
      const R gneq = gs - cv2r * rt;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R qn = qa[a] - rho_ * u[a] * (m.U + R(D + 2) * th);
        qn -= R(2) * (pn[a][0] * u[0] + pn[a][1] * u[1] + pn[a][2] * u[2]);
        qn -= u[a] * trp;
        m.qf[a] = (a < D) ? qn : R(0);
        m.qg[a] = (a < D) ? ga[a] - cv2r * th * rho_ * u[a] - u[a] * gneq : R(0);
      }
      // tau_q = 1/2 + (tau - 1/2) / Pr
      m.omq = R(1) / (R(0.5) + R(p.tau_m_half * p.inv_pr) / (rho_ * th));
    }
    (void)Ef; (void)G; (void)Ed;
    return m;
  };

  // xh_q . q_g: the g quasi-equilibrium's term is w_q times this
  auto qe_g = [&](auto qc, const Mom& m) -> R {
    constexpr int q = decltype(qc)::value;
    R ag = R(0);
    if constexpr (S::moves(q, 0)) ag = fma(R(S::xh(q, 0)), m.qg[0], ag);
    if constexpr (S::moves(q, 1)) ag = fma(R(S::xh(q, 1)), m.qg[1], ag);
    if constexpr (D == 3 && S::moves(q, 2)) ag = fma(R(S::xh(q, 2)), m.qg[2], ag);
    return ag;
  };
  (void)qe_g;

  if constexpr (is_step(MODE)) {
    Mom mc[RO];
#pragma unroll
    for (int r = 0; r < RO; ++r) mc[r] = moments(r);
    // Float compute: the set's constants rounded to float give sum_i w_i xh_i xh_i
    // = (1 + m) I with |m| ~ 1e-8, which BGK with omega near 2 would turn
    // into a steady drift of the momentum (and in the compressible model of
    // the energy).  The missing equilibrium momentum rho m' u~ (m' = 1/(1+m) - 1)
    // is restored as w_i rho m' (xh_i . u~) and the missing energy as w_i dE / sum w,
    // both added to the small non-equilibrium difference f^eq - f before it is
    // scaled by omega, where they are far above its rounding.  Neither changes the
    // other invariants (odd/even symmetry of the set).
    // 16-bit storage rounds far above these defects: no energy restoration there.
    // The compressible model's Hermite terms (|u~|^2 up to ~6 at Ma 2) also carry
    // the rounded even moments into the equilibrium's mass, sum_i w_i rho P_i =
    // rho (1 + S) + (rho - 1) d0 with S, d0 ~ 1e-8 (peq_mass_defect): restored as
    // w_i cM in the same non-equilibrium difference, cM = -(rho S + (rho - 1) d0)
    // (sum_i w_i = 1 up to d0), and its energy cM sum_i w_i |xh_i|^2 counted in
    // the energy balance after the small residual E_pre - E_eq has formed (added
    // to the accumulator first it would fall below half an ulp of its terms).
    constexpr bool EFIX = COMP && DEV && !TR::coarse;
    R Eeq[RO], cM[RO];
#pragma unroll
    for (int r = 0; r < RO; ++r) {
      Eeq[r] = R(0);
      cM[r] = R(0);
      if constexpr (EFIX) {
        const Mom& m = mc[r];
        cM[r] = -fma(m.rho, peq_mass_defect<D, R>(p.mdef, m.ux, m.uy, m.uz, m.U, m.eta), m.dr * R(p.mdef[0]));
      }
    }
    // populations outer, cells inner: each population's store address is set up once
    static_for<Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr double X = S::xh(q, 0) * S::xh(q, 0) + S::xh(q, 1) * S::xh(q, 1) + S::xh(q, 2) * S::xh(q, 2);
      const R w = R(S::w(q));
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        if (D == 2 && r >= ovalid) break;
        const Mom& m = mc[r];
        R a = R(0);
        if constexpr (S::moves(q, 0)) a = fma(R(S::xh(q, 0)), m.ux, a);
        if constexpr (S::moves(q, 1)) a = fma(R(S::xh(q, 1)), m.uy, a);
        if constexpr (D == 3 && S::moves(q, 2)) a = fma(R(S::xh(q, 2)), m.uz, a);
        const R pm1 = peq_minus1<N, D, COMP, R>(a, m.U, m.eta, R(X));
        R feq_dev;  // f^eq - w = w ((rho - 1) + rho (P - 1)) (DEV), or f^eq
        if constexpr (DEV) feq_dev = fma(w * m.rho, pm1, w * m.dr);
        else feq_dev = w * m.rho * (R(1) + pm1);
        // f* = f + omega (f^eq - f): the small non-equilibrium part carries the rounding
        R df = feq_dev - ft[q][r];
        if constexpr (DEV && X != 0.0) df = fma(w * (m.rho * R(p.cmom1)), a, df);
        if constexpr (EFIX) df = fma(w, cM[r], df);
        R fo = fma(m.omega, df, ft[q][r]);
        if constexpr (MODE == MODE_STEP_QE) {
          // + (omega - omega_q)(f* - f^eq): the quasi-equilibrium's heat-flux term
          constexpr double kf = S::w(q) * (X - (D + 2)) / (2.0 * (D + 2));
          R aq = R(0);
          if constexpr (S::moves(q, 0)) aq = fma(R(S::xh(q, 0)), m.qf[0], aq);
          if constexpr (S::moves(q, 1)) aq = fma(R(S::xh(q, 1)), m.qf[1], aq);
          if constexpr (D == 3 && S::moves(q, 2)) aq = fma(R(S::xh(q, 2)), m.qf[2], aq);
          fo = fma((m.omega - m.omq) * R(kf), aq, fo);
        }
        put_at(q, r, SUBREF ? fo + w : fo);
        if constexpr (COMP) {
          R geq;
          if constexpr (DEV) geq = cv2 * fma(m.theta, feq_dev, m.eta * w);
          else geq = cv2 * m.theta * feq_dev;
          if constexpr (EFIX) {
            if constexpr (X != 0.0) Eeq[r] = fma(R(X), feq_dev, Eeq[r]);
            Eeq[r] += geq;
            ft[q][r] = geq - ft[Q + q][r];  // f_q is stored: its register keeps g^eq - g
          } else {
            R go = fma(m.omega, geq - ft[Q + q][r], ft[Q + q][r]);
            if constexpr (MODE == MODE_STEP_QE) go = fma((m.omega - m.omq) * w, qe_g(qc, m), go);
            put_at(Q + q, r, SUBREF ? go + cv2 * w : go);
          }
        }
      }
    });
    if constexpr (EFIX) {
      R cE[RO];
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        cE[r] = ((mc[r].Epre - Eeq[r]) - cM[r] * R(p.swX)) * R(1.0 / p.sw);
      }
      static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const R w = R(S::w(q));
#pragma unroll
        for (int r = 0; r < RO; ++r) {
          if (D == 2 && r >= ovalid) break;
          R go = fma(mc[r].omega, fma(w, cE[r], ft[q][r]), ft[Q + q][r]);
          if constexpr (MODE == MODE_STEP_QE) go = fma((mc[r].omega - mc[r].omq) * w, qe_g(qc, mc[r]), go);
          put_at(Q + q, r, SUBREF ? go + cv2 * w : go);
        }
      });
    }
  } else {
#pragma unroll
    for (int r = 0; r < RO; ++r) {
      if (r >= ovalid) break;
      auto put = [&](int k, R v) { put_at(k, r, v); };
      const int lc = lc_of(r), rowb = rowb_of(r);
      auto get_lam = [&](int k) -> R {
        if constexpr (D == 3)
          return TR::ldb(make_rsrc(lam_in + int64_t(k) * p.pstride, p.pstride), boff<E>(lc), rowb);
        else
          return TR::ld(at(lam_in + int64_t(k) * p.pstride, lc));
      };
      if constexpr (MODE == MODE_ADJ_STREAM) {
        static_for<Q>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          put(q, ft[q][r]);
        });
      } else {
        const Mom mm = moments(r);
        const R ux = mm.ux, uy = mm.uy, uz = mm.uz, U = mm.U;
      // adjoint of the weakly compressible collision at this cell
      R lm[Q];
      if constexpr (MODE == MODE_ADJ_COLLIDE) {
        static_for<Q>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          lm[q] = get_lam(q);
        });
      } else {
        static_for<Q>([&](auto qc) {
          constexpr int q = decltype(qc)::value;
          lm[q] = lam[q][r];
        });
      }
      const R omega = R(p.omega);
      R v0 = R(0), vx = R(0), vy = R(0), vz = R(0);
      static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        R a = R(0);
        if constexpr (S::moves(q, 0)) a = fma(R(S::xh(q, 0)), ux, a);
        if constexpr (S::moves(q, 1)) a = fma(R(S::xh(q, 1)), uy, a);
        if constexpr (D == 3 && S::moves(q, 2)) a = fma(R(S::xh(q, 2)), uz, a);
        R Pq, Pa, PU;
        peq_derivs<N, R>(a, U, Pq, Pa, PU);
        const R lw = lm[q] * R(S::w(q));
        v0 = fma(lw, Pq - Pa * a - R(2) * PU * U, v0);
        const R c2 = R(2) * PU;
        if constexpr (S::moves(q, 0)) vx = fma(lw, Pa * R(S::xh(q, 0)), vx);
        if constexpr (S::moves(q, 1)) vy = fma(lw, Pa * R(S::xh(q, 1)), vy);
        if constexpr (D == 3 && S::moves(q, 2)) vz = fma(lw, Pa * R(S::xh(q, 2)), vz);
        // the 2 P_U u~ part of d f^eq / d j~ is common to every direction
        vx = fma(lw * c2, ux, vx);
        vy = fma(lw * c2, uy, vy);
        if constexpr (D == 3) vz = fma(lw * c2, uz, vz);
      });
      const R om1 = R(1) - omega;
      static_for<Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        R m = v0;
        if constexpr (S::moves(q, 0)) m = fma(R(S::xh(q, 0)), vx, m);
        if constexpr (S::moves(q, 1)) m = fma(R(S::xh(q, 1)), vy, m);
        if constexpr (D == 3 && S::moves(q, 2)) m = fma(R(S::xh(q, 2)), vz, m);
        const R mu = fma(om1, lm[q], omega * m);
        put(q, mu);
      });
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Per-cell kernels: equilibrium initialisation, moments, loss / init adjoints
// ---------------------------------------------------------------------------

struct CellParams {
  const void* f;      // populations (storage type)
  void* out_f;        // populations out (init)
  const void* rho;    // [cells] compute type
  const void* u;      // [D][cells]
  const void* theta;  // [cells] or null
  const void* lam;    // [Q][cells] compute type
  void* out_rho;
  void* out_u;
  void* out_theta;
  double* partial;    // [nblocks][NPART] block sums of the moments kernel
  int64_t ncell;
  int nblocks;        // blocks of the moments kernel (grid-stride loop)
  double cs;          // u = cs * u~
  double cv2mD, inv2cv, sw, swX, swx[3];
  double scale;       // 1 / ncell (KE adjoint)
};

template <int SET, int N, int A, int ST>
__global__ __launch_bounds__(256) void init_kernel(CellParams p) {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  constexpr int D = S::D, Q = S::Q;
  constexpr bool COMP = (A == 2);
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= p.ncell) return;
  const R* rho_p = static_cast<const R*>(p.rho);
  const R* u_p = static_cast<const R*>(p.u);
  const R* th_p = static_cast<const R*>(p.theta);
  E* out = static_cast<E*>(p.out_f);
  const R rho = rho_p[e];
  const R inv_cs = R(1.0 / p.cs);
  const R ux = u_p[e] * inv_cs, uy = u_p[p.ncell + e] * inv_cs;
  const R uz = (D == 3) ? u_p[2 * p.ncell + e] * inv_cs : R(0);
  const R U = ux * ux + uy * uy + uz * uz;
  const R theta = (COMP && th_p) ? th_p[e] : R(1);
  const R eta = theta - R(1);
  static_for<Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr double X = S::xh(q, 0) * S::xh(q, 0) + S::xh(q, 1) * S::xh(q, 1) + S::xh(q, 2) * S::xh(q, 2);
    const R a = R(S::xh(q, 0)) * ux + R(S::xh(q, 1)) * uy + R(S::xh(q, 2)) * uz;
    const R pm1 = peq_minus1<N, D, COMP, R>(a, U, eta, R(X));
    const R w = R(S::w(q));
    R fe;
    if constexpr (TR::dev) fe = w * fma(rho - R(1), R(1) + pm1, pm1);
    else fe = w * rho * (R(1) + pm1);
    constexpr bool whole = TR::dev && !TR::stores_dev;  // deviation arithmetic, whole values stored
    TR::st(out + int64_t(q) * p.ncell + e, whole ? fe + w : fe);
    if constexpr (COMP) {
      R ge;
      if constexpr (TR::dev) ge = R(p.cv2mD) * fma(theta, fe, eta * w);
      else ge = R(p.cv2mD) * theta * fe;
      TR::st(out + int64_t(Q + q) * p.ncell + e, whole ? ge + R(p.cv2mD) * w : ge);
    }
  });
}

// Per-cell moments of a stored state plus block partial sums:
// [0] mass, [1..3] momentum, [4] sum |u|^2/2, [5] energy, [6] min rho,
// [7] min theta, [8] count of non-finite cells.  Grid-stride loop.
constexpr int NPART = 9;

template <int SET, int A, int ST>
__global__ __launch_bounds__(256) void moments_kernel(CellParams p) {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  constexpr int D = S::D, Q = S::Q;
  constexpr bool COMP = (A == 2);
  const E* f = static_cast<const E*>(p.f);
  R* orho = static_cast<R*>(p.out_rho);
  R* ou = static_cast<R*>(p.out_u);
  R* oth = static_cast<R*>(p.out_theta);
  double acc[NPART] = {0, 0, 0, 0, 0, 0, 1e300, 1e300, 0};
  for (int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x; e < p.ncell; e += int64_t(gridDim.x) * 256) {
    double rho = 0, jx = 0, jy = 0, jz = 0, Ef = 0, G = 0;
    static_for<Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      double v = double(TR::ld(f + int64_t(q) * p.ncell + e));
      if constexpr (TR::stores_dev) v += S::w(q);
      rho += v;
      jx += S::xh(q, 0) * v;
      jy += S::xh(q, 1) * v;
      jz += S::xh(q, 2) * v;
      constexpr double X = S::xh(q, 0) * S::xh(q, 0) + S::xh(q, 1) * S::xh(q, 1) + S::xh(q, 2) * S::xh(q, 2);
      Ef += X * v;
      if constexpr (COMP) {
        double gv = double(TR::ld(f + int64_t(Q + q) * p.ncell + e));
        if constexpr (TR::stores_dev) gv += p.cv2mD * S::w(q);
        G += gv;
      }
    });
    const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const double U = ux * ux + uy * uy + uz * uz;
    const double theta = COMP ? (Ef - rho * U + G) * p.inv2cv / rho : 1.0;
    const double cs = p.cs;
    if (orho) orho[e] = R(rho);
    if (ou) {
      ou[e] = R(cs * ux);
      ou[p.ncell + e] = R(cs * uy);
      if (D == 3) ou[2 * p.ncell + e] = R(cs * uz);
    }
    if (oth) oth[e] = R(theta);
    const bool finite = isfinite(rho) && isfinite(U) && isfinite(theta);
    if (!finite) {
      acc[8] += 1.0;
      continue;
    }
    acc[0] += rho;
    acc[1] += rho * cs * ux;
    acc[2] += rho * cs * uy;
    acc[3] += rho * cs * uz;
    acc[4] += 0.5 * cs * cs * U;
    acc[5] += 0.5 * (Ef + G);
    acc[6] = fmin(acc[6], rho);
    acc[7] = fmin(acc[7], theta);
  }
  // block reduction (deterministic order)
  __shared__ double red[NPART][256];
#pragma unroll
  for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < NPART; ++k) {
        if (k == 6 || k == 7) red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        else red[k][threadIdx.x] += red[k][threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NPART) p.partial[int64_t(blockIdx.x) * NPART + threadIdx.x] = red[threadIdx.x][0];
}

// Final reduction of the block partials (one block).
static __global__ __launch_bounds__(256) void reduce_partials_kernel(const double* partial, int nblocks, double* out) {
  __shared__ double red[NPART][256];
  double acc[NPART] = {0, 0, 0, 0, 0, 0, 1e300, 1e300, 0};
  for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
      const double v = partial[int64_t(b) * NPART + k];
      if (k == 6 || k == 7) acc[k] = fmin(acc[k], v);
      else acc[k] += v;
    }
  }
#pragma unroll
  for (int k = 0; k < NPART; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < NPART; ++k) {
        if (k == 6 || k == 7) red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
        else red[k][threadIdx.x] += red[k][threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < NPART) out[threadIdx.x] = red[threadIdx.x][0];
}

// lam_k = dK/df_k, K = (1/ncell) sum |u|^2/2, u = cs j~/rho:
// lam_k = scale * cs^2 * u~ . (xh_k - u~) / rho
template <int SET, int ST>
__global__ __launch_bounds__(256) void ke_adjoint_kernel(CellParams p) {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  using E = typename TR::elem;
  constexpr int D = S::D, Q = S::Q;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= p.ncell) return;
  const E* f = static_cast<const E*>(p.f);
  R* lam = static_cast<R*>(p.out_f);
  R rho = R(0), jx = R(0), jy = R(0), jz = R(0);
  static_for<Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const R v = TR::ld(f + int64_t(q) * p.ncell + e) + (TR::stores_dev ? R(S::w(q)) : R(0));
    rho += v;
    jx = fma(R(S::xh(q, 0)), v, jx);
    jy = fma(R(S::xh(q, 1)), v, jy);
    jz = fma(R(S::xh(q, 2)), v, jz);
  });
  const R ux = jx / rho, uy = jy / rho, uz = (D == 3) ? jz / rho : R(0);
  const R c = R(p.scale * p.cs * p.cs) / rho;
  const R uu = ux * ux + uy * uy + uz * uz;
  static_for<Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const R a = R(S::xh(q, 0)) * ux + R(S::xh(q, 1)) * uy + R(S::xh(q, 2)) * uz;
    lam[int64_t(q) * p.ncell + e] = c * (a - uu);
  });
}

// grad_u = sum_k lam_k d f^eq_k / d u, with d f^eq/d u = (w rho / cs)(P_a xh + 2 P_U u~)
template <int SET, int N, int ST>
__global__ __launch_bounds__(256) void init_adjoint_kernel(CellParams p) {
  using S = Set<SET>;
  using TR = StoreT<ST>;
  using R = typename TR::real;
  constexpr int D = S::D, Q = S::Q;
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= p.ncell) return;
  const R* rho_p = static_cast<const R*>(p.rho);
  const R* u_p = static_cast<const R*>(p.u);
  const R* lam = static_cast<const R*>(p.lam);
  R* gu = static_cast<R*>(p.out_u);
  const R inv_cs = R(1.0 / p.cs);
  const R ux = u_p[e] * inv_cs, uy = u_p[p.ncell + e] * inv_cs;
  const R uz = (D == 3) ? u_p[2 * p.ncell + e] * inv_cs : R(0);
  const R U = ux * ux + uy * uy + uz * uz;
  R gx = R(0), gy = R(0), gz = R(0);
  static_for<Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    const R a = R(S::xh(q, 0)) * ux + R(S::xh(q, 1)) * uy + R(S::xh(q, 2)) * uz;
    R Pq, Pa, PU;
    peq_derivs<N, R>(a, U, Pq, Pa, PU);
    const R lw = lam[int64_t(q) * p.ncell + e] * R(S::w(q));
    gx = fma(lw, Pa * R(S::xh(q, 0)) + R(2) * PU * ux, gx);
    gy = fma(lw, Pa * R(S::xh(q, 1)) + R(2) * PU * uy, gy);
    gz = fma(lw, Pa * R(S::xh(q, 2)) + R(2) * PU * uz, gz);
  });
  const R c = rho_p[e] * inv_cs;
  gu[e] = c * gx;
  gu[p.ncell + e] = c * gy;
  if (D == 3) gu[2 * p.ncell + e] = c * gz;
}

}  // namespace lbm
