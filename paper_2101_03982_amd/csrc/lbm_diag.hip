// Enstrophy E = <|curl u|^2> of a velocity field on the uniform periodic grid
// (the diagnostic of Sec. 4.2), by central differences:
//   d f / d x_a (x) ~ sum_{j=1..m} c_j (f(x + j e_a) - f(x - j e_a)) / dx.
// 3D: one node per thread, neighbours read through the caches;
// 2D: one wave per grid row.  FP64 arithmetic on the loaded values,
// block sums in a fixed tree order, then one block adds the block sums in
// index order: the result does not depend on scheduling.
#include <algorithm>

#include "lbm_diag.hpp"

namespace lbm {
namespace {

constexpr int DIAG_THREADS = 256;
constexpr int MAX_HALF_WIDTH = 4;

struct CurlParams {
  const void* u;
  int64_t n[3];   // nx, ny, nz
  int64_t ncell;
  int m;          // half-width of the stencil
  double c[MAX_HALF_WIDTH];  // c_j / dx
  double* partial;
};

// Index of i + d on a periodic line of N nodes, |d| <= MAX_HALF_WIDTH.
__device__ inline int64_t wrap(int64_t i, int d, int64_t N) {
  int64_t k = i + d;
  if (k >= N || k < 0) {
    k %= N;
    if (k < 0) k += N;
  }
  return k;
}

// Central difference of field f along the line through node `row + i*stride`
// (row = the node's index with its coordinate along this axis set to 0).
template <typename R>
__device__ inline double ddx(const R* f, int64_t row, int64_t i, int64_t N, int64_t stride, const CurlParams& p) {
  double s = 0.0;
  for (int j = 1; j <= p.m; ++j) {
    const double fp = double(f[row + wrap(i, j, N) * stride]);
    const double fm = double(f[row + wrap(i, -j, N) * stride]);
    s = fma(p.c[j - 1], fp - fm, s);
  }
  return s;
}

// 2D: one wave per grid row y at a time, its lanes along x (the row's
// coordinate is found once per row), so every neighbour-row load is coalesced.
constexpr int DIAG_WAVES = DIAG_THREADS / 64;

template <typename R>
__global__ __launch_bounds__(DIAG_THREADS) void enstrophy2d_kernel(CurlParams p) {
  const R* u = static_cast<const R*>(p.u);
  const R* ux = u;
  const R* uy = u + p.ncell;
  const int64_t nx = p.n[0], ny = p.n[1];
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int64_t y = int64_t(blockIdx.x) * DIAG_WAVES + (threadIdx.x >> 6); y < ny; y += int64_t(gridDim.x) * DIAG_WAVES) {
    const int64_t rowbase = y * nx;  // index of node (0, y)
    for (int64_t x = lane; x < nx; x += 64) {
      const double wz = ddx(uy, rowbase, x, nx, 1, p) - ddx(ux, x, y, ny, nx, p);
      acc += wz * wz;
    }
  }
  __shared__ double red[DIAG_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.partial[blockIdx.x] = red[0];
}

// 3D: one node per thread, 64 x 4 (x, y) tiles of one z plane, every
// neighbour read straight from global memory through the caches (8 M loads
// per node, re-read from L1 and L2; nothing waits on a barrier).  Lanes past
// a ragged edge load nothing.  FP32 at 128^3: 34.6 us with 32-bit indices,
// 46.6 us with 64-bit ones, against 61.0 us for tiles marching along z with
// LDS planes and a register window along z (their loads waited on the
// tile's barriers).
constexpr int ZT_X = 64, ZT_Y = DIAG_WAVES;

__device__ inline int64_t wrap_any(int64_t i, int64_t N) {
  if (i >= 0 && i < N) return i;
  i %= N;
  return i < 0 ? i + N : i;
}

// i + d on a periodic line of N nodes, |d| <= MAX_HALF_WIDTH, i in [0, N):
// one add or subtract of N unless the line is shorter than the stencil
template <typename I>
__device__ inline I wrap_near(I i, int d, I N) {
  I k = i + d;
  k += (k < 0) ? N : 0;
  k -= (k >= N) ? N : 0;
  return (k >= 0 && k < N) ? k : I(wrap_any(k, N));
}

// I: the index type, 32-bit when all three components hold fewer than 2^31
// elements (the host's choice), else 64-bit
template <typename R, int M, typename I>
__global__ __launch_bounds__(DIAG_THREADS) void enstrophy3d_kernel(CurlParams p) {
  const R* u = static_cast<const R*>(p.u);
  const R* ux = u;
  const R* uy = u + p.ncell;
  const R* uz = u + 2 * p.ncell;
  const I nx = I(p.n[0]), ny = I(p.n[1]), nz = I(p.n[2]);
  const I tiles_x = (nx + ZT_X - 1) / ZT_X, tiles_y = (ny + ZT_Y - 1) / ZT_Y;
  const int64_t tiles = int64_t(tiles_x) * tiles_y * nz;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double c[M];
#pragma unroll
  for (int j = 0; j < M; ++j) c[j] = p.c[j];
  double acc = 0.0;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const I tt = I(t), tx = tt % tiles_x, ty = (tt / tiles_x) % tiles_y, z = tt / (tiles_x * tiles_y);
    const I x = tx * ZT_X + lane, y = ty * ZT_Y + wv;
    if (x >= nx || y >= ny) continue;
    const I row = (z * ny + y) * nx;  // node (0, y, z)
    double dxuy = 0, dxuz = 0, dyux = 0, dyuz = 0, dzux = 0, dzuy = 0;
#pragma unroll
    for (int j = 1; j <= M; ++j) {
      const double cj = c[j - 1];
      const I xp = row + wrap_near(x, j, nx), xm = row + wrap_near(x, -j, nx);
      const I yp = (z * ny + wrap_near(y, j, ny)) * nx + x, ym = (z * ny + wrap_near(y, -j, ny)) * nx + x;
      const I zp = (wrap_near(z, j, nz) * ny + y) * nx + x, zm = (wrap_near(z, -j, nz) * ny + y) * nx + x;
      dxuy = fma(cj, double(uy[xp]) - double(uy[xm]), dxuy);
      dxuz = fma(cj, double(uz[xp]) - double(uz[xm]), dxuz);
      dyux = fma(cj, double(ux[yp]) - double(ux[ym]), dyux);
      dyuz = fma(cj, double(uz[yp]) - double(uz[ym]), dyuz);
      dzux = fma(cj, double(ux[zp]) - double(ux[zm]), dzux);
      dzuy = fma(cj, double(uy[zp]) - double(uy[zm]), dzuy);
    }
    const double ox = dyuz - dzuy, oy = dzux - dxuz, oz = dxuy - dyux;
    acc += ox * ox + oy * oy + oz * oz;
  }
  __shared__ double red[DIAG_THREADS];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) p.partial[blockIdx.x] = red[0];
}

template <typename R, typename I>
void launch_3d_idx(const CurlParams& p, int blocks, hipStream_t s) {
  switch (p.m) {
    case 1: hipLaunchKernelGGL((enstrophy3d_kernel<R, 1, I>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    case 2: hipLaunchKernelGGL((enstrophy3d_kernel<R, 2, I>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    case 3: hipLaunchKernelGGL((enstrophy3d_kernel<R, 3, I>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    default: hipLaunchKernelGGL((enstrophy3d_kernel<R, 4, I>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
  }
}

template <typename R>
void launch_3d(const CurlParams& p, int blocks, hipStream_t s) {
  const int64_t tiles = ((p.n[0] + ZT_X - 1) / ZT_X) * ((p.n[1] + ZT_Y - 1) / ZT_Y) * p.n[2];
  if (3 * p.ncell < (int64_t(1) << 31) && tiles < (int64_t(1) << 31))
    launch_3d_idx<R, int32_t>(p, blocks, s);
  else
    launch_3d_idx<R, int64_t>(p, blocks, s);
}

__global__ __launch_bounds__(DIAG_THREADS) void sum_blocks_kernel(const double* partial, int nblocks, double* out) {
  __shared__ double red[DIAG_THREADS];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += DIAG_THREADS) acc += partial[b];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t launch_enstrophy(const void* u, bool f64, const int64_t n[3], int D, int m, const double* coef,
                            double* partial, int max_blocks, double* result, hipStream_t s) {
  if (m < 1 || m > MAX_HALF_WIDTH || max_blocks < 1 || (D != 2 && D != 3)) return hipErrorInvalidValue;
  CurlParams p{};
  p.u = u;
  for (int a = 0; a < 3; ++a) p.n[a] = n[a];
  p.ncell = n[0] * n[1] * n[2];
  p.m = m;
  for (int j = 0; j < m; ++j) p.c[j] = coef[j];
  p.partial = partial;
  // 3D: one block per (x, y) tile of a plane, up to eight blocks per compute
  // unit (2048; then each block takes every 2048th tile: the single-block
  // sum of 8192 partials at 128^3 took 9.9 us against 5 us); 2D: one wave
  // per row
  const int64_t want = (D == 3) ? std::min<int64_t>(((n[0] + ZT_X - 1) / ZT_X) * ((n[1] + ZT_Y - 1) / ZT_Y) * n[2], 2048)
                                : (n[1] * n[2] + DIAG_WAVES - 1) / DIAG_WAVES;
  const int blocks = want < 1 ? 1 : int(want < max_blocks ? want : max_blocks);
  if (f64) {
    if (D == 3) launch_3d<double>(p, blocks, s);
    else hipLaunchKernelGGL((enstrophy2d_kernel<double>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
  } else {
    if (D == 3) launch_3d<float>(p, blocks, s);
    else hipLaunchKernelGGL((enstrophy2d_kernel<float>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(DIAG_THREADS), 0, s, partial, blocks, result);
  return hipGetLastError();
}

}  // namespace lbm
