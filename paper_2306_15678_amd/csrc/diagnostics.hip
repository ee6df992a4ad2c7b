// diagnostics.hip -- hot-area count and spatial moments of a fluence.
//
// Hot areas (Results: a hot area is a closed region of the fluence with
// w >= w_p, N_ha their number): 4-connected components of the thresholded
// FP64 array, optionally continuing across the periodic window edge.
// Labelling is a lock-free union-find over pixel indices: every hot pixel
// starts as its own root, parents only ever decrease (device-scope
// atomicMin), so L[x] <= x holds throughout and every walk to a root ends;
// a union retries only after lowering one of its two labels.  Then a
// compression pass points every pixel at its root and the roots are
// counted with fixed-order partial sums.
//
// Moments (Eq. (8) family): Q(p, m) = sum w^p (x^2 + y^2)^m dx^2 on the
// cell-centred grid, FP64 partial sums per block, summed on the host in
// block order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"

// Device scratch of the allocation-free hot-area count: labels of an n x n
// grid with n <= kStaticMaxN, the overflow flag and the per-block partial
// counts.  One copy per GPU, held until the process ends; host code never
// uses this name as an address (it stands for a host-side shadow): the
// device address comes from hipGetSymbolAddress in static_scratch().
static __device__ __align__(256) unsigned char scratch[ssfm::kStaticScratchBytes];

namespace ssfm {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    // with device dev current: that device's copy of the array
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

namespace {

constexpr int kUniteCap = 1 << 22;  // far above any chain on a 4096^2 grid

__device__ __forceinline__ int load_label(const int* lab, int x) {
  return __hip_atomic_load(lab + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of hot pixel x (labels only decrease along a walk).
__device__ __forceinline__ int find_root(const int* lab, int x) {
  int p = load_label(lab, x);
  while (p != x) {
    x = p;
    p = load_label(lab, x);
  }
  return x;
}

__device__ __forceinline__ void unite(int* lab, int a, int b, int* overflow) {
  for (int it = 0; it < kUniteCap; ++it) {
    a = find_root(lab, a);
    b = find_root(lab, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    // link the larger root b under a; if b was no longer a root, continue
    // from its (smaller) parent
    const int old = atomicMin(lab + b, a);
    if (old == b) return;
    b = old;
  }
  *overflow = 1;
}

// Deterministic reduction of NV doubles over a 256-thread block (sum or
// max); valid in thread 0.  red: shared [4][NV].
template <int NV, int THREADS, bool MAX>
__device__ __forceinline__ void block_reduce_diag(double (&v)[NV], double* red) {
  for (int off = 32; off >= 1; off >>= 1)
    for (int k = 0; k < NV; ++k) {
      const double o = __shfl_xor(v[k], off, 64);
      v[k] = MAX ? fmax(v[k], o) : v[k] + o;
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) {
      double t = red[k];
      for (int q = 1; q < THREADS / 64; ++q) t = MAX ? fmax(t, red[q * NV + k]) : t + red[q * NV + k];
      v[k] = t;
    }
}

__global__ void k_set_i32(int* p, int v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) p[0] = v;
}

__global__ void k_hot_init(const double* __restrict__ w, int64_t n2, double thr,
                           int* __restrict__ lab) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x)
    lab[i] = (w[i] >= thr) ? int(i) : -1;
}

__global__ void k_hot_merge(int* lab, int n, int periodic, int* overflow) {
  const int64_t n2 = int64_t(n) * n;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (load_label(lab, int(i)) < 0) continue;
    const int y = int(i / n), x = int(i - int64_t(y) * n);
    // right and down neighbours (wrapping when periodic)
    int xr = x + 1, yd = y + 1;
    if (xr == n) xr = periodic ? 0 : -1;
    if (yd == n) yd = periodic ? 0 : -1;
    if (xr >= 0) {
      const int j = y * n + xr;
      if (load_label(lab, j) >= 0) unite(lab, int(i), j, overflow);
    }
    if (yd >= 0) {
      const int j = yd * n + x;
      if (load_label(lab, j) >= 0) unite(lab, int(i), j, overflow);
    }
  }
}

__global__ void k_hot_compress(int* lab, int64_t n2) {
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    if (load_label(lab, int(i)) < 0) continue;
    const int r = find_root(lab, int(i));
    __hip_atomic_store(lab + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Per-block count of roots (lab[i] == i), one double per block.
__global__ void __launch_bounds__(256) k_hot_count(const int* __restrict__ lab, int64_t n2,
                                                   double* part) {
  __shared__ double red[4];
  double c = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x)
    c += (lab[i] == int(i)) ? 1.0 : 0.0;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_moment(const double* __restrict__ w, int n, double dx,
                                                double p, int m, double* part) {
  __shared__ double red[4];
  const int64_t n2 = int64_t(n) * n;
  const bool p1 = (p == 1.0), p2 = (p == 2.0);
  double s = 0.0;
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int y = int(i / n), x = int(i - int64_t(y) * n);
    const double xc = (x + 0.5 - n / 2.0) * dx, yc = (y + 0.5 - n / 2.0) * dx;
    const double r2 = xc * xc + yc * yc;
    double rm = 1.0;
    for (int k = 0; k < m; ++k) rm *= r2;
    const double wi = w[i];
    const double wp = p1 ? wi : (p2 ? wi * wi : pow(wi, p));
    s += wp * rm;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Per-block FP64 partials of the measure vector's sums over an n x n
// fluence: [sum w, sum w r^2, sum w^2, sum w^2 r^2, max w] (grid-stride,
// then a fixed tree per block).
__global__ void __launch_bounds__(256) k_measure(const double* __restrict__ w, int n, double dx,
                                                 double* part) {
  __shared__ double red[4 * 5];
  const int64_t n2 = int64_t(n) * n;
  double s[4] = {0.0, 0.0, 0.0, 0.0}, mx[1] = {0.0};
  for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n2;
       i += int64_t(gridDim.x) * blockDim.x) {
    const int y = int(i / n), x = int(i - int64_t(y) * n);
    const double xc = (x + 0.5 - n / 2.0) * dx, yc = (y + 0.5 - n / 2.0) * dx;
    const double r2 = xc * xc + yc * yc;
    const double wi = w[i], w2 = wi * wi;
    s[0] += wi;
    s[1] += wi * r2;
    s[2] += w2;
    s[3] += w2 * r2;
    mx[0] = fmax(mx[0], wi);
  }
  block_reduce_diag<4, 256, false>(s, red);
  block_reduce_diag<1, 256, true>(mx, red + 16);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) part[5 * blockIdx.x + k] = s[k];
    part[5 * blockIdx.x + 4] = mx[0];
  }
}

}  // namespace

hipError_t launch_measure(const double* w, int n, double dx, double* part, int n_part,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_measure, dim3(n_part), dim3(256), 0, s, w, n, dx, part);
  return hipGetLastError();
}

hipError_t launch_hot_areas(const double* w, int n, double threshold, int periodic, int* labels,
                            int* overflow, double* part, int n_part, hipStream_t s) {
  const int64_t n2 = int64_t(n) * n;
  const int grid = int(std::min<int64_t>((n2 + 255) / 256, 8192));
  hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, s, overflow, 0);
  hipLaunchKernelGGL(k_hot_init, dim3(grid), dim3(256), 0, s, w, n2, threshold, labels);
  hipLaunchKernelGGL(k_hot_merge, dim3(grid), dim3(256), 0, s, labels, n, periodic, overflow);
  hipLaunchKernelGGL(k_hot_compress, dim3(grid), dim3(256), 0, s, labels, n2);
  hipLaunchKernelGGL(k_hot_count, dim3(n_part), dim3(256), 0, s, labels, n2, part);
  return hipGetLastError();
}

hipError_t launch_moment(const double* w, int n, double dx, double p, int m, double* part,
                         int n_part, hipStream_t s) {
  hipLaunchKernelGGL(k_moment, dim3(n_part), dim3(256), 0, s, w, n, dx, p, m, part);
  return hipGetLastError();
}

}  // namespace ssfm
