// Dense reconstruction C x_1 U_1 ... x_p U_p (eq. (reconstructed), Sec. 2.2) from
// factors the caller holds on the device, for callers that cannot allocate device
// memory: the intermediates of the n-mode product chain live in a fixed array of this
// library (`scratch`), so the call allocates nothing.
//
// In host code `scratch` names a host-side stand-in, not a device address: its device
// address is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that pointer is handed to kernels. Each GPU holds its own copy of
// the array until the process ends; calls that overlap on one GPU race for it.
#include "tdb_common.h"
#include "tdb_kernels.h"
#include "noalloc.h"

#include <mutex>

namespace tdb {

static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Y[a, o, b] = sum_i U[o * r + i] X[a, i, b] for X of dims (A, r, B) and U row-major
// N x r: the n-mode product with one basis (FP64 arithmetic, output in TY).
template <typename TY>
__global__ void __launch_bounds__(256) k_na_ttm(const double* __restrict__ X, const double* __restrict__ U,
                                                TY* __restrict__ Y, long long A, int r, int N, long long B) {
  const long long total = A * (long long)N * B;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += stride) {
    const long long b = idx % B;
    const long long t = idx / B;
    const int o = (int)(t % N);
    const long long a = t / N;
    const double* xp = X + a * (long long)r * B + b;
    const double* up = U + (long long)o * r;
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc += up[i] * xp[(long long)i * B];
    Y[idx] = (TY)acc;
  }
}

template <typename TY>
hipError_t launch_na_ttm(const double* X, const double* U, TY* Y, long long A, int r, int N, long long B,
                         hipStream_t s) {
  const long long total = A * (long long)N * B;
  long long blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_na_ttm<TY>, dim3((unsigned)blocks), dim3(256), 0, s, X, U, Y, A, r, N, B);
  return hipGetLastError();
}

// The device address of `scratch` on the current device, looked up on the first call
// made with that device current.
static hipError_t scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

NoallocPlan noalloc_plan(int p, const long long* dims, const int* ranks) {
  NoallocPlan pl{};
  pl.p = p;
  // contract the modes in order of increasing N_n / r_n (ties by mode), so that the
  // intermediates stay small; the last product writes the output
  for (int k = 0; k < p; ++k) pl.order[k] = k;
  for (int i = 1; i < p; ++i)
    for (int j = i; j > 0; --j) {
      const int x = pl.order[j - 1], y = pl.order[j];
      const double rx = (double)dims[x] / ranks[x], ry = (double)dims[y] / ranks[y];
      if (rx > ry || (rx == ry && x > y)) { pl.order[j - 1] = y; pl.order[j] = x; } else break;
    }
  long long cd[TDB_P];
  for (int k = 0; k < p; ++k) cd[k] = ranks[k];
  pl.max_inter = 0;
  for (int q = 0; q + 1 < p; ++q) {
    cd[pl.order[q]] = dims[pl.order[q]];
    long long sz = 1;
    for (int k = 0; k < p; ++k) sz *= cd[k];
    if (sz > pl.max_inter) pl.max_inter = sz;
  }
  return pl;
}

hipError_t noalloc_reconstruct(const NoallocPlan& pl, const long long* dims, const int* ranks, const double* C,
                               const double* const* U, int out_f32, void* out, hipStream_t s) {
  double* base = nullptr;
  hipError_t e = scratch_on_current_device(&base);
  if (e != hipSuccess) return e;
  double* half[2] = {base, base + NOALLOC_SCRATCH_DOUBLES / 2};
  const int p = pl.p;
  long long cd[TDB_P];
  for (int k = 0; k < p; ++k) cd[k] = ranks[k];
  const double* in = C;
  for (int q = 0; q < p; ++q) {
    const int k = pl.order[q];
    long long A = 1, B = 1;
    for (int j = 0; j < k; ++j) A *= cd[j];
    for (int j = k + 1; j < p; ++j) B *= cd[j];
    if (q + 1 < p) {
      double* o = half[q & 1];
      e = launch_na_ttm<double>(in, U[k], o, A, (int)cd[k], (int)dims[k], B, s);
      in = o;
    } else if (out_f32) {
      e = launch_na_ttm<float>(in, U[k], static_cast<float*>(out), A, (int)cd[k], (int)dims[k], B, s);
    } else {
      e = launch_na_ttm<double>(in, U[k], static_cast<double*>(out), A, (int)cd[k], (int)dims[k], B, s);
    }
    if (e != hipSuccess) return e;
    cd[k] = dims[k];
  }
  return hipSuccess;
}

}  // namespace tdb
