// Enstrophy E = <|curl u|^2> of a velocity field on the uniform periodic grid
// (the diagnostic of Sec. 4.2), by central differences:
//   d f / d x_a (x) ~ sum_{j=1..m} c_j (f(x + j e_a) - f(x - j e_a)) / dx.
// 3D: tiles marching along z (register window for z, LDS plane for x and y);
// 2D: one wave per grid row.  FP64 arithmetic on the loaded values,
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

// 3D: a 64 x 4 (x, y) tile marching through ZT_Z planes of z (4: enough
// blocks to fill the chip at 128^3; measured faster than 8 or 16).  The z
// derivatives come from a window of 2M + 1 planes kept in registers per
// thread (u_x, u_y); the x and y derivatives from one plane staged in LDS with
// its halo (u_x with a y halo, u_y with an x halo, u_z with both).  About ten
// loads per node instead of the 12 M of the row kernel.  Every load index is
// wrapped onto the periodic grid; lanes past a ragged edge load wrapped
// nodes and add nothing.
constexpr int ZT_X = 64, ZT_Y = DIAG_WAVES, ZT_Z = 4;

__device__ inline int64_t wrap_any(int64_t i, int64_t N) {
  if (i >= 0 && i < N) return i;
  i %= N;
  return i < 0 ? i + N : i;
}

template <typename R, int M>
__global__ __launch_bounds__(DIAG_THREADS) void enstrophy3d_kernel(CurlParams p) {
  const R* u = static_cast<const R*>(p.u);
  const R* ux = u;
  const R* uy = u + p.ncell;
  const R* uz = u + 2 * p.ncell;
  const int64_t nx = p.n[0], ny = p.n[1], nz = p.n[2], nxy = nx * ny;
  const int64_t tiles_x = (nx + ZT_X - 1) / ZT_X, tiles_y = (ny + ZT_Y - 1) / ZT_Y;
  const int64_t tiles = tiles_x * tiles_y * ((nz + ZT_Z - 1) / ZT_Z);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __shared__ R sx[ZT_Y + 2 * M][ZT_X];          // u_x, rows y - M .. y + 3 + M
  __shared__ R sy[ZT_Y][ZT_X + 2 * M];          // u_y, columns x - M .. x + 63 + M
  __shared__ R sz[ZT_Y + 2 * M][ZT_X + 2 * M];  // u_z, both halos
  double c[M];
#pragma unroll
  for (int j = 0; j < M; ++j) c[j] = p.c[j];
  double acc = 0.0;
  for (int64_t t = blockIdx.x; t < tiles; t += gridDim.x) {
    const int64_t tx = t % tiles_x, ty = (t / tiles_x) % tiles_y, tz = t / (tiles_x * tiles_y);
    const int64_t x0 = tx * ZT_X, y0 = ty * ZT_Y, z0 = tz * ZT_Z;
    const int64_t z1 = (z0 + ZT_Z < nz) ? z0 + ZT_Z : nz;
    const bool valid = (x0 + lane < nx) && (y0 + wv < ny);
    const int64_t col = wrap_any(y0 + wv, ny) * nx + wrap_any(x0 + lane, nx);  // (x, y) of this thread
    // window: w[k] = u(z + k - M), k = 0 .. 2M; the last slot is loaded per plane
    R wx[2 * M + 1], wy[2 * M + 1];
#pragma unroll
    for (int k = 0; k < 2 * M; ++k) {
      const int64_t e = wrap_any(z0 + k - M, nz) * nxy + col;
      wx[k] = ux[e];
      wy[k] = uy[e];
    }
    for (int64_t z = z0; z < z1; ++z) {
      const int64_t plane = z * nxy;
      {
        const int64_t e = wrap_any(z + M, nz) * nxy + col;
        wx[2 * M] = ux[e];
        wy[2 * M] = uy[e];
      }
      __syncthreads();  // the previous plane's reads of the LDS buffers are done
      for (int i = threadIdx.x; i < (ZT_Y + 2 * M) * ZT_X; i += DIAG_THREADS) {
        const int r = i / ZT_X, q = i % ZT_X;
        sx[r][q] = ux[plane + wrap_any(y0 + r - M, ny) * nx + wrap_any(x0 + q, nx)];
      }
      for (int i = threadIdx.x; i < ZT_Y * (ZT_X + 2 * M); i += DIAG_THREADS) {
        const int r = i / (ZT_X + 2 * M), q = i % (ZT_X + 2 * M);
        sy[r][q] = uy[plane + wrap_any(y0 + r, ny) * nx + wrap_any(x0 + q - M, nx)];
      }
      for (int i = threadIdx.x; i < (ZT_Y + 2 * M) * (ZT_X + 2 * M); i += DIAG_THREADS) {
        const int r = i / (ZT_X + 2 * M), q = i % (ZT_X + 2 * M);
        sz[r][q] = uz[plane + wrap_any(y0 + r - M, ny) * nx + wrap_any(x0 + q - M, nx)];
      }
      __syncthreads();
      double dxuy = 0, dxuz = 0, dyux = 0, dyuz = 0, dzux = 0, dzuy = 0;
#pragma unroll
      for (int j = 1; j <= M; ++j) {
        const double cj = c[j - 1];
        dxuy = fma(cj, double(sy[wv][lane + M + j]) - double(sy[wv][lane + M - j]), dxuy);
        dxuz = fma(cj, double(sz[wv + M][lane + M + j]) - double(sz[wv + M][lane + M - j]), dxuz);
        dyux = fma(cj, double(sx[wv + M + j][lane]) - double(sx[wv + M - j][lane]), dyux);
        dyuz = fma(cj, double(sz[wv + M + j][lane + M]) - double(sz[wv + M - j][lane + M]), dyuz);
        dzux = fma(cj, double(wx[M + j]) - double(wx[M - j]), dzux);
        dzuy = fma(cj, double(wy[M + j]) - double(wy[M - j]), dzuy);
      }
      if (valid) {
        const double ox = dyuz - dzuy, oy = dzux - dxuz, oz = dxuy - dyux;
        acc += ox * ox + oy * oy + oz * oz;
      }
#pragma unroll
      for (int k = 0; k < 2 * M; ++k) {
        wx[k] = wx[k + 1];
        wy[k] = wy[k + 1];
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

template <typename R>
void launch_3d(const CurlParams& p, int blocks, hipStream_t s) {
  switch (p.m) {
    case 1: hipLaunchKernelGGL((enstrophy3d_kernel<R, 1>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    case 2: hipLaunchKernelGGL((enstrophy3d_kernel<R, 2>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    case 3: hipLaunchKernelGGL((enstrophy3d_kernel<R, 3>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
    default: hipLaunchKernelGGL((enstrophy3d_kernel<R, 4>), dim3(blocks), dim3(DIAG_THREADS), 0, s, p); break;
  }
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
  // 3D: one block per tile of the z-marching kernel; 2D: one wave per row
  const int64_t want = (D == 3) ? ((n[0] + ZT_X - 1) / ZT_X) * ((n[1] + ZT_Y - 1) / ZT_Y) * ((n[2] + ZT_Z - 1) / ZT_Z)
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
