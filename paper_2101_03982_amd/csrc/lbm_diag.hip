// Enstrophy E = <|curl u|^2> of a velocity field on the uniform periodic grid
// (the diagnostic of Sec. 4.2), by central differences:
//   d f / d x_a (x) ~ sum_{j=1..m} c_j (f(x + j e_a) - f(x - j e_a)) / dx.
// One wave per grid row (lanes along x), FP64 arithmetic on the loaded values,
// block sums in a fixed tree order, then one block adds the block sums in
// index order: the result does not depend on scheduling.
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

// One wave per grid row (y, z) at a time, its lanes along x: the row's
// coordinates are found once per row (uniform), and every load of a
// neighbour row is a coalesced row access.
constexpr int DIAG_WAVES = DIAG_THREADS / 64;

template <typename R, int D>
__global__ __launch_bounds__(DIAG_THREADS) void enstrophy_kernel(CurlParams p) {
  const R* u = static_cast<const R*>(p.u);
  const R* ux = u;
  const R* uy = u + p.ncell;
  const R* uz = u + 2 * p.ncell;
  const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2], nxy = nx * ny;
  const int lane = threadIdx.x & 63;
  const int64_t rows = ny * nz;
  double acc = 0.0;
  for (int64_t row = int64_t(blockIdx.x) * DIAG_WAVES + (threadIdx.x >> 6); row < rows;
       row += int64_t(gridDim.x) * DIAG_WAVES) {
    const int64_t y = row % ny, z = row / ny;
    const int64_t rowbase = row * nx;  // index of node (0, y, z)
    for (int64_t x = lane; x < nx; x += 64) {
      const int64_t e = rowbase + x;
      const int64_t ry = e - y * nx, rz = e - z * nxy;
      if constexpr (D == 3) {
        const double wx = ddx(uz, ry, y, ny, nx, p) - ddx(uy, rz, z, nz, nxy, p);
        const double wy = ddx(ux, rz, z, nz, nxy, p) - ddx(uz, rowbase, x, nx, 1, p);
        const double wz = ddx(uy, rowbase, x, nx, 1, p) - ddx(ux, ry, y, ny, nx, p);
        acc += wx * wx + wy * wy + wz * wz;
      } else {
        const double wz = ddx(uy, rowbase, x, nx, 1, p) - ddx(ux, ry, y, ny, nx, p);
        acc += wz * wz;
      }
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
  const int64_t want = (n[1] * n[2] + DIAG_WAVES - 1) / DIAG_WAVES;  // one wave per row
  const int blocks = want < 1 ? 1 : int(want < max_blocks ? want : max_blocks);
  if (f64) {
    if (D == 3) hipLaunchKernelGGL((enstrophy_kernel<double, 3>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
    else hipLaunchKernelGGL((enstrophy_kernel<double, 2>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
  } else {
    if (D == 3) hipLaunchKernelGGL((enstrophy_kernel<float, 3>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
    else hipLaunchKernelGGL((enstrophy_kernel<float, 2>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_blocks_kernel, dim3(1), dim3(DIAG_THREADS), 0, s, partial, blocks, result);
  return hipGetLastError();
}

}  // namespace lbm
