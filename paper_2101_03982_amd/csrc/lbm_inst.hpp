// Instantiation of the built kernels of one (velocity set, storage, stencil
// length) and their launcher table.  Each generated unit under _build/
// instantiates one such part, so that the parts compile in parallel.
#pragma once

#include <algorithm>

#include "lbm_dispatch.hpp"

namespace lbm {

template <class F, int... I>
inline void host_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
inline void host_for(F&& f) {
  host_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Blocks of one sl_kernel instantiation that fit on a compute unit at once.
template <int SET, int NS, int N, int A, int ST, int MODE, int CP, int XP>
int blocks_per_cu() {
  using TL = Tile<SET, NS, A, ST, cells_per_thread<Set<SET>::D, Set<SET>::Q, A, ST, MODE>()>;
  static const int per_cu = [] {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&sl_kernel<SET, NS, N, A, ST, MODE, CP, XP>),
                                                     TL::NT, 0) != hipSuccess || nb < 1)
      nb = 1;
    return nb;
  }();
  return per_cu;
}

// Whether a kernel interpolates along x through LDS at all (3D with a stencil
// longer than one node): only those have the single-load variant XP = 0.
template <int SET, int NS>
constexpr bool has_x_pairs() {
  return Set<SET>::D == 3 && NS > 1;
}

template <int SET, int NS, int N, int A, int ST, int MODE, int CP = 0>
hipError_t launch_step(const KParams& p, hipStream_t s) {
  using E = typename StoreT<ST>::elem;
  constexpr int D = Set<SET>::D;
  constexpr int RO = cells_per_thread<D, Set<SET>::Q, A, ST, MODE>();
  using TL = Tile<SET, NS, A, ST, RO>;
  KParams q = p;
  q.tiles[0] = (p.n[0] + TL::TX - 1) / TL::TX;
  if (D == 3) {
    q.tiles[1] = (p.n[1] + TL::NW - 1) / TL::NW;
    q.tiles[2] = (p.n[2] + RO - 1) / RO;
  } else {
    q.tiles[1] = (p.n[1] + TL::NW * RO - 1) / (TL::NW * RO);
    q.tiles[2] = 1;
  }
  // x pairs in one two-element load: x periodic with nx even (a pair never
  // straddles the wrap or a row end) and every buffer the interpolation reads
  // aligned to two elements
  auto al2 = [](const void* ptr) { return reinterpret_cast<uintptr_t>(ptr) % (2 * sizeof(E)) == 0; };
  constexpr bool reads_src = MODE != MODE_ADJ_STREAM;
  constexpr bool reads_src2 = MODE == MODE_ADJ_STEP || MODE == MODE_ADJ_STREAM;
  const bool pairs = p.bc[0] == 0 && (p.n[0] & 1) == 0 && (p.pstride & 1) == 0 && (!reads_src || al2(p.src)) &&
                     (!reads_src2 || al2(p.src2));
  const int per_cu = (has_x_pairs<SET, NS>() && !pairs) ? blocks_per_cu<SET, NS, N, A, ST, MODE, CP, 0>()
                                                         : blocks_per_cu<SET, NS, N, A, ST, MODE, CP, 1>();
  const int64_t ntiles = int64_t(q.tiles[0]) * q.tiles[1] * q.tiles[2];
  q.chunk = int((ntiles + 7) / 8);
  q.rsy = q.rsz = 0;
  q.by = q.bz = 0;
  if (D == 3) {  // one (y, z) block of tiles per XCD
    // 4 x 2 (y, z) blocks: an XCD's z neighbours of a tile then come within
    // the tiles it holds at once (measured against 2 x 4: D3Q45 f + g 256^3
    // FP32 4 % and BF16 2 % faster, the 27-velocity sets 4-7 % at 256^3 and
    // equal at 128^3); 2 x 4 for tiles one cell thick, whose brick order
    // below was measured with it
    q.ysl = (RO == 1) ? 1 : 2;
    q.rsy = (q.tiles[1] + (1 << q.ysl) - 1) >> q.ysl;
    q.rsz = (q.tiles[2] + (8 >> q.ysl) - 1) / (8 >> q.ysl);
    q.chunk = q.tiles[0] * q.rsy * q.rsz;
    // tiles one cell thick along z (RO = 1): bricks when the XCD's xy plane
    // of tiles is larger than half the blocks it holds at once (sl_kernel).
    // Measured on D3Q45 f + g at 256^3: FP64 15 % faster than the x, y, z
    // order (11.75 against 13.79 ms); with two cells per thread (the FP32 and
    // 16-bit kernels) the x, y, z order reads less (16-bit: 2.6x the state
    // against 3.9x) and runs 2 % faster, so they keep it.
    const int window = per_cu * (p.cus > 0 ? p.cus / 8 : 32);
    if (RO == 1 && 2 * q.tiles[0] * q.rsy > window) {
      q.bz = std::min(q.rsz, 16);
      int by = 1;
      while (2 * by * q.bz <= window && 2 * by <= q.rsy) by *= 2;
      q.by = by;
      const int nby = (q.rsy + q.by - 1) / q.by, nbz = (q.rsz + q.bz - 1) / q.bz;
      q.chunk = q.tiles[0] * nby * nbz * q.by * q.bz;
    }
  }
  const dim3 grid(unsigned(q.chunk) * 8u);
  // stochastic rounding: its own instantiation of the 16-bit step kernels
  constexpr bool has_sr = (ST == ST_BF16 || ST == ST_F16) && MODE == MODE_STEP;
  const bool sr = has_sr && p.sr != 0;
  if constexpr (has_x_pairs<SET, NS>()) {
    if (!pairs) {
      if constexpr (has_sr) {
        if (sr) {
          hipLaunchKernelGGL((sl_kernel<SET, NS, N, A, ST, MODE, CP, 0, 1>), grid, dim3(TL::NT), 0, s, q);
          return hipGetLastError();
        }
      }
      hipLaunchKernelGGL((sl_kernel<SET, NS, N, A, ST, MODE, CP, 0>), grid, dim3(TL::NT), 0, s, q);
      return hipGetLastError();
    }
  }
  if constexpr (has_sr) {
    if (sr) {
      hipLaunchKernelGGL((sl_kernel<SET, NS, N, A, ST, MODE, CP, 1, 1>), grid, dim3(TL::NT), 0, s, q);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((sl_kernel<SET, NS, N, A, ST, MODE, CP, 1>), grid, dim3(TL::NT), 0, s, q);
  return hipGetLastError();
}

inline dim3 cell_grid(int64_t ncell) { return dim3(unsigned((ncell + 255) / 256)); }

template <int SET, int N, int A, int ST>
hipError_t launch_init(const CellParams& p, hipStream_t s) {
  hipLaunchKernelGGL((init_kernel<SET, N, A, ST>), cell_grid(p.ncell), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int SET, int A, int ST>
hipError_t launch_moments(const CellParams& p, hipStream_t s) {
  hipLaunchKernelGGL((moments_kernel<SET, A, ST>), dim3(unsigned(p.nblocks)), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int SET, int ST>
hipError_t launch_ke_adjoint(const CellParams& p, hipStream_t s) {
  hipLaunchKernelGGL((ke_adjoint_kernel<SET, ST>), cell_grid(p.ncell), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int SET, int N, int ST>
hipError_t launch_init_adjoint(const CellParams& p, hipStream_t s) {
  hipLaunchKernelGGL((init_adjoint_kernel<SET, N, ST>), cell_grid(p.ncell), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <int SET, int ST, int NS>
bool find_kernels_part(int order, int arrays, Kernels* out) {
  bool found = false;
  host_for<3>([&](auto nc) {
    constexpr int N = decltype(nc)::value + 2;
    host_for<2>([&](auto ac) {
      constexpr int A = decltype(ac)::value + 1;
      if constexpr (combo_built<SET, NS, N, A, ST>()) {
        if (order == N && arrays == A) {
          found = true;
          *out = Kernels{};
          out->mode[MODE_STEP] = &launch_step<SET, NS, N, A, ST, MODE_STEP>;
          if constexpr (Set<SET>::D == 3 && NS == 4)
            out->step_stream = &launch_step<SET, NS, N, A, ST, MODE_STEP, CP_STREAM>;
          if constexpr (mode_built<SET, NS, N, A, ST, MODE_STEP_QE>()) {
            out->step_qe = &launch_step<SET, NS, N, A, ST, MODE_STEP_QE>;
            if constexpr (Set<SET>::D == 3 && NS == 4)
              out->step_qe_stream = &launch_step<SET, NS, N, A, ST, MODE_STEP_QE, CP_STREAM>;
          }
          if constexpr (mode_built<SET, NS, N, A, ST, MODE_ADJ_COLLIDE>()) {
            out->mode[MODE_ADJ_COLLIDE] = &launch_step<SET, NS, N, A, ST, MODE_ADJ_COLLIDE>;
            out->mode[MODE_ADJ_STEP] = &launch_step<SET, NS, N, A, ST, MODE_ADJ_STEP>;
            out->mode[MODE_ADJ_STREAM] = &launch_step<SET, NS, N, A, ST, MODE_ADJ_STREAM>;
            out->ke_adjoint = &launch_ke_adjoint<SET, ST>;
            out->init_adjoint = &launch_init_adjoint<SET, N, ST>;
          }
          out->init = &launch_init<SET, N, A, ST>;
          out->moments = &launch_moments<SET, A, ST>;
        }
      }
    });
  });
  return found;
}

}  // namespace lbm
