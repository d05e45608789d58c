// Host-side view of the kernels built for one velocity set: launchers looked
// up by (stencil length, Hermite order, number of population arrays, storage).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_kernels.hpp"

namespace lbm {

using StepLaunch = hipError_t (*)(const KParams&, hipStream_t);
using CellLaunch = hipError_t (*)(const CellParams&, hipStream_t);

struct Kernels {
  StepLaunch mode[4] = {nullptr, nullptr, nullptr, nullptr};  // indexed by Mode
  // the forward step with non-temporal result stores (3D sets, n = 4 only)
  StepLaunch step_stream = nullptr;
  // the compressible forward step with the Pr != 1 quasi-equilibrium (and its
  // streamed-store copy)
  StepLaunch step_qe = nullptr, step_qe_stream = nullptr;
  CellLaunch init = nullptr;
  CellLaunch moments = nullptr;     // writes partials; grid = CellParams::nblocks
  CellLaunch ke_adjoint = nullptr;
  CellLaunch init_adjoint = nullptr;
};

// Blocks of the moments kernel: at most MOMENT_BLOCKS, and no more than one
// per 256 cells.
constexpr int MOMENT_BLOCKS = 1024;
inline int moment_blocks(int64_t ncell) {
  const int64_t b = (ncell + 255) / 256;
  return int(b < MOMENT_BLOCKS ? (b < 1 ? 1 : b) : MOMENT_BLOCKS);
}

// The paper's cell-wise support (p = 4, the order of all its runs) is built for
// the weakly compressible sets of its Taylor-Green study and D2Q9, in FP64
// and FP32, forward step only.
constexpr int GLC_P4 = GLC_BASE + 4;
template <int SET, int ST>
constexpr bool glc_built() {
  return (SET == D2Q9 || SET == D3Q13 || SET == D3Q21 || SET == D3Q27 || SET == D3V27) &&
         (ST == ST_F64 || ST == ST_F32);
}

// Which combinations are compiled.  Every set gets the forward step for each
// stencil length 2..5 (1: the on-lattice copy, D2Q9 and D3Q27 only).
// Hermite orders: N = 2 everywhere; N = 3 for the degree-7 set (D3V27); N = 4
// for the degree-9 sets.  The compressible model (two arrays) uses N = 4.
// 16-bit deviation storage: the 3D sets at their workload order (N = 2,
// N = 3 for D3V27) and D3Q45 compressible.  Adjoint modes: FP64/FP32, weakly
// compressible, N = 2.
template <int SET, int NS, int N, int A, int ST>
constexpr bool combo_built() {
  constexpr int D = Set<SET>::D;
  constexpr int deg = Set<SET>::degree;
  if (2 * N > deg) return false;
  if constexpr (Support<NS>::glc) return glc_built<SET, ST>() && A == 1 && N == (deg == 7 ? 3 : 2);
  if (N == 3 && deg != 7) return false;
  if (A == 2 && N != 4) return false;
  if (NS == 1 && !(SET == D2Q9 || SET == D3Q27)) return false;
  if (ST == ST_BF16 || ST == ST_F16) {
    if (D != 3) return false;
    if (SET == D3Q45) return A == 2;
    return A == 1 && N == (deg == 7 ? 3 : 2);
  }
  return true;
}

template <int SET, int NS, int N, int A, int ST, int MODE>
constexpr bool mode_built() {
  if (!combo_built<SET, NS, N, A, ST>()) return false;
  if (MODE == MODE_STEP) return true;
  if (Support<NS>::glc) return false;
  // the Pr != 1 quasi-equilibrium: the compressible workloads' sets and stencils, FP64 / FP32
  if (MODE == MODE_STEP_QE)
    return A == 2 && (ST == ST_F64 || ST == ST_F32) &&
           ((SET == D3Q45 && NS == 4) || ((SET == D2Q19 || SET == D2Q25) && NS == 5));
  return A == 1 && N == 2 && (ST == ST_F64 || ST == ST_F32);
}

// Which (set, storage, stencil length) parts exist as compiled units.
template <int SET, int ST, int NS>
constexpr bool part_exists() {
  if (Support<NS>::glc) return glc_built<SET, ST>();
  if (NS == 1 && !(SET == D2Q9 || SET == D3Q27)) return false;
  if ((ST == ST_BF16 || ST == ST_F16) && Set<SET>::D != 3) return false;
  return true;
}

template <int SET, int ST, int NS>
bool find_kernels_part(int order, int arrays, Kernels* out);

// Launcher table of a set (defined in the host library, dispatching to the
// per-set instantiation units).
bool find_kernels(int set, int ns, int order, int arrays, int storage, Kernels* out);

}  // namespace lbm
