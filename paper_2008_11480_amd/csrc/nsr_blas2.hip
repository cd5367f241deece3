// HBM-bound kernels of the solver: norms for the scalar preconditioner
// (Section 2), the implicit G_0 = I / alpha, and the Richardson mat-vecs
// r = b - A theta and theta += G r (eq. redttk1).  All reductions go through
// per-block partials reduced in a fixed order, so results are deterministic.
#include "nsr_internal.h"

namespace nsr {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double out = 0.0;
  if (threadIdx.x == 0) out = (red[0] + red[1]) + (red[2] + red[3]);
  return out;
}

// One block per 'rows_per_block' rows; sum of squares of the block's rows.
constexpr int kRowsPerBlock = 8;

__global__ void __launch_bounds__(kThreads)
sumsq_kernel(const double* __restrict__ A, int64_t lda, int64_t n, double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  double s = 0.0;
  for (int rr = 0; rr < kRowsPerBlock; ++rr) {
    const int64_t row = r0 + rr;
    if (row >= n) break;
    const double* a = A + row * lda;
    for (int64_t c = threadIdx.x; c < n; c += kThreads) {
      const double v = a[c];
      s += v * v;
    }
  }
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// One wave per row: rowsum[row] = sum_j |A[row][j]|.
__global__ void __launch_bounds__(kThreads)
rowabs_kernel(const double* __restrict__ A, int64_t lda, int64_t n, double* __restrict__ rowsum) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* a = A + row * lda;
  double s = 0.0;
  for (int64_t c = lane; c < n; c += 64) s += fabs(a[c]);
  s = wave_sum(s);
  if (lane == 0) rowsum[row] = s;
}

// Single block, fixed order: out = sum / max / sqrt(sum) of partial[0..count).
__global__ void __launch_bounds__(kThreads)
reduce_kernel(const double* __restrict__ partial, int64_t count, double* __restrict__ out, int mode,
              double eps) {
  __shared__ double sh[kThreads];
  const bool is_max = (mode == 1 || mode == 3);
  double v = is_max ? -INFINITY : 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kThreads) {
    const double x = partial[i];
    v = is_max ? fmax(v, x) : v + x;
  }
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sh[threadIdx.x], b = sh[threadIdx.x + w];
      sh[threadIdx.x] = is_max ? fmax(a, b) : a + b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double r = sh[0];
    if (mode == 2) r = sqrt(r);
    if (mode == 3) r = 0.5 * r + eps;   // ||A||_inf / 2 + eps
    out[0] = r;
  }
}

// F = I - A / alpha (computed in float64, stored as T, optional bf16 copy),
// sum of F^2 per block (one block per kRowsPerBlock rows).
template <typename T>
__global__ void __launch_bounds__(kThreads)
init_resid_kernel(const double* __restrict__ A, int64_t lda, int64_t n,
                  const double* __restrict__ alpha, const double* __restrict__ sdiag,
                  T* __restrict__ F, int64_t ldf, uint16_t* __restrict__ Fb,
                  double* __restrict__ partial) {
  __shared__ double red[4];
  const double inv = 1.0 / alpha[0];
  const int64_t r0 = (int64_t)blockIdx.x * kRowsPerBlock;
  double s = 0.0;
  // Each thread loads kEw elements (and their S entries) before it stores
  // them: loads and stores share one in-order completion counter, so a load
  // issued after a store waits for it.
  constexpr int kEw = 8;
  for (int rr = 0; rr < kRowsPerBlock; ++rr) {
    const int64_t row = r0 + rr;
    if (row >= n) break;
    for (int64_t c0 = threadIdx.x; c0 < n; c0 += (int64_t)kThreads * kEw) {
      double a[kEw], sd[kEw];
#pragma unroll
      for (int u = 0; u < kEw; ++u) {
        const int64_t c = c0 + (int64_t)u * kThreads;
        a[u] = c < n ? A[row * lda + c] : 0.0;
        sd[u] = (sdiag && c < n) ? sdiag[c] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < kEw; ++u) {
        const int64_t c = c0 + (int64_t)u * kThreads;
        if (c >= n) break;
        double v = sdiag ? -a[u] / sd[u] : -a[u] * inv;
        if (c == row) v += 1.0;
        const T t = (T)v;
        F[row * ldf + c] = t;
        if (Fb) Fb[row * ldf + c] = __builtin_bit_cast(uint16_t, (__bf16)(float)t);
        s += (double)t * (double)t;
      }
    }
  }
  const double tt = block_sum(s, red);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = tt;
}

// G = (I + C) / alpha  (C may be null).
template <typename T>
__global__ void __launch_bounds__(kThreads)
scaled_identity_plus_kernel(const T* __restrict__ C, int64_t ldc, int64_t n,
                            const double* __restrict__ alpha, const double* __restrict__ sdiag,
                            T* __restrict__ G, int64_t ldg) {
  const int64_t row = blockIdx.y;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= n || c >= n) return;
  const double inv = 1.0 / (sdiag ? sdiag[row] : alpha[0]);
  double v = C ? (double)C[row * ldc + c] : 0.0;
  if (c == row) v += 1.0;
  G[row * ldg + c] = (T)(v * inv);
}

// D = X + Y element-wise (n x n, common leading dimension; D may alias X or
// Y), with an optional bf16 copy of D.
template <typename T>
__global__ void __launch_bounds__(kThreads)
add_kernel(const T* X, const T* Y, T* D, uint16_t* Db, int64_t ld, int64_t n) {
  const int64_t row = blockIdx.y;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= n || c >= n) return;
  const int64_t i = row * ld + c;
  const T v = X[i] + Y[i];
  D[i] = v;
  if (Db) Db[i] = __builtin_bit_cast(uint16_t, (__bf16)(float)v);
}

// hist_f[k] = scal[1] (||F_k||_F), hist_r[k - 1] = scal[2] (||r||_2): the
// per-step history of a captured iteration, read back once at the end.
__global__ void record_kernel(const double* __restrict__ scal, double* __restrict__ hist_f,
                              double* __restrict__ hist_r, int k) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hist_f[k] = scal[1];
    hist_r[k - 1] = scal[2];
  }
}

// sdiag[i] = A_ii; neg[i] = -A_ii (a max-reduction of neg gives -min A_ii).
__global__ void __launch_bounds__(kThreads)
diag_kernel(const double* __restrict__ A, int64_t lda, int64_t n, double* __restrict__ sdiag,
            double* __restrict__ neg) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double v = A[i * lda + i];
  sdiag[i] = v;
  neg[i] = -v;
}

// dst (float64 or float32) = (T) src, n x n.
template <typename S, typename D>
__global__ void __launch_bounds__(kThreads)
convert_kernel(const S* __restrict__ src, int64_t lds, int64_t n, D* __restrict__ dst, int64_t ldd) {
  const int64_t row = blockIdx.y;
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (row >= n || c >= n) return;
  dst[row * ldd + c] = (D)src[row * lds + c];
}

template <typename T> struct Pair;
template <> struct Pair<double> { typedef double2 type; };
template <> struct Pair<float> { typedef float2 type; };

// Dot product of one matrix row with x (float64 accumulate), by one wave,
// lane-partial (the caller reduces over the wave).  vec: the row and x are
// read two elements per lane (16-byte row loads for float64), two chunks of
// 128 columns in flight with separate partial sums; needs the row and x
// aligned to two elements.
template <typename T>
__device__ __forceinline__ double row_dot(const T* __restrict__ a, const double* __restrict__ x,
                                          int64_t n, bool vec) {
  const int lane = threadIdx.x & 63;
  double s0 = 0.0, s1 = 0.0;
  if (vec) {
    typedef typename Pair<T>::type P;
    const int64_t n2 = n & ~(int64_t)1;
    int64_t c = 2 * lane;
    for (; c + 128 < n2; c += 256) {
      const P a0 = *reinterpret_cast<const P*>(a + c);
      const P a1 = *reinterpret_cast<const P*>(a + c + 128);
      const double2 x0 = *reinterpret_cast<const double2*>(x + c);
      const double2 x1 = *reinterpret_cast<const double2*>(x + c + 128);
      s0 += (double)a0.x * x0.x + (double)a0.y * x0.y;
      s1 += (double)a1.x * x1.x + (double)a1.y * x1.y;
    }
    if (c < n2) {
      const P a0 = *reinterpret_cast<const P*>(a + c);
      const double2 x0 = *reinterpret_cast<const double2*>(x + c);
      s0 += (double)a0.x * x0.x + (double)a0.y * x0.y;
    }
    if ((n & 1) && lane == 0) s1 += (double)a[n - 1] * x[n - 1];
  } else {
    for (int64_t c = lane; c < n; c += 64) s0 += (double)a[c] * x[c];
  }
  return s0 + s1;
}

// r = b - A theta: one wave per row, 4 rows per block; partial sum of r^2.
__global__ void __launch_bounds__(kThreads)
gemv_resid_kernel(const double* __restrict__ A, int64_t lda, int64_t n,
                  const double* __restrict__ b, const double* __restrict__ theta,
                  double* __restrict__ r, double* __restrict__ partial, int vec) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  double rv = 0.0;
  if (row < n) {
    double s = row_dot(A + row * lda, theta, n, vec != 0);
    s = wave_sum(s);
    rv = b[row] - s;
    if (lane == 0) r[row] = rv;
  }
  if (lane == 0) red[wave] = rv * rv;
  __syncthreads();
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// theta += G r: one wave per row (G float64 or float32, float64 accumulate).
template <typename T>
__global__ void __launch_bounds__(kThreads)
gemv_update_kernel(const T* __restrict__ G, int64_t ldg, int64_t n,
                   const double* __restrict__ r, double* __restrict__ theta, int vec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= n) return;
  double s = row_dot(G + row * ldg, r, n, vec != 0);
  s = wave_sum(s);
  if (lane == 0) theta[row] += s;
}

// y = M x + z (z may be null), or y += M x + z with accumulate: one wave per
// row, float64 accumulation (M float64 or float32).
template <typename T>
__global__ void __launch_bounds__(kThreads)
gemv_kernel(const T* __restrict__ M, int64_t ldm, int64_t n, const double* __restrict__ x,
            const double* __restrict__ z, double* __restrict__ y, int accumulate, int vec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= n) return;
  double s = row_dot(M + row * ldm, x, n, vec != 0);
  s = wave_sum(s);
  if (lane == 0) {
    if (z) s += z[row];
    y[row] = accumulate ? y[row] + s : s;
  }
}

__global__ void __launch_bounds__(kThreads)
vec_scale_kernel(const double* __restrict__ b, const double* __restrict__ alpha,
                 const double* __restrict__ sdiag, double* __restrict__ theta, int64_t n,
                 int accumulate) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const double v = b[i] / (sdiag ? sdiag[i] : alpha[0]);
  theta[i] = accumulate ? theta[i] + v : v;
}

__global__ void __launch_bounds__(kThreads)
vec_sumsq_kernel(const double* __restrict__ v, int64_t n, double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    s += v[i] * v[i];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

}  // namespace

int64_t sumsq_partials(int64_t n) { return (n + kRowsPerBlock - 1) / kRowsPerBlock; }
int64_t gemv_partials(int64_t n) { return (n + 3) / 4; }

// Rows of M (leading dimension ld) and the vector x can be read two elements
// at a time: every row starts on a two-element boundary.
template <typename T>
bool pair_aligned(const T* M, int64_t ld, const double* x) {
  return (ld % 2) == 0 && (reinterpret_cast<uintptr_t>(M) % (2 * sizeof(T))) == 0 &&
         (reinterpret_cast<uintptr_t>(x) % 16) == 0;
}

int64_t launch_sumsq(const double* A, int64_t lda, int64_t n, double* partial, hipStream_t st) {
  const int64_t nb = sumsq_partials(n);
  hipLaunchKernelGGL(sumsq_kernel, dim3((unsigned)nb), dim3(kThreads), 0, st, A, lda, n, partial);
  return nb;
}

void launch_rowabs(const double* A, int64_t lda, int64_t n, double* rowsum, hipStream_t st) {
  hipLaunchKernelGGL(rowabs_kernel, dim3((unsigned)((n + 3) / 4)), dim3(kThreads), 0, st, A, lda,
                     n, rowsum);
}

void launch_reduce(const double* partial, int64_t count, double* out, int mode, double eps,
                   hipStream_t st) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, st, partial, count, out, mode, eps);
}

template <typename T>
int64_t launch_init_resid(const double* A, int64_t lda, int64_t n, const double* alpha,
                          const double* sdiag, T* F, int64_t ldf, uint16_t* Fb, double* partial,
                          hipStream_t st) {
  const int64_t nb = sumsq_partials(n);
  hipLaunchKernelGGL(init_resid_kernel<T>, dim3((unsigned)nb), dim3(kThreads), 0, st, A, lda, n,
                     alpha, sdiag, F, ldf, Fb, partial);
  return nb;
}
template int64_t launch_init_resid<double>(const double*, int64_t, int64_t, const double*,
                                           const double*, double*, int64_t, uint16_t*, double*,
                                           hipStream_t);
template int64_t launch_init_resid<float>(const double*, int64_t, int64_t, const double*,
                                          const double*, float*, int64_t, uint16_t*, double*,
                                          hipStream_t);

template <typename T>
void launch_scaled_identity_plus(const T* C, int64_t ldc, int64_t n, const double* alpha,
                                 const double* sdiag, T* G, int64_t ldg, hipStream_t st) {
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)n);
  hipLaunchKernelGGL(scaled_identity_plus_kernel<T>, grid, dim3(kThreads), 0, st, C, ldc, n, alpha,
                     sdiag, G, ldg);
}
template void launch_scaled_identity_plus<double>(const double*, int64_t, int64_t, const double*,
                                                  const double*, double*, int64_t, hipStream_t);
template void launch_scaled_identity_plus<float>(const float*, int64_t, int64_t, const double*,
                                                 const double*, float*, int64_t, hipStream_t);

void launch_record(const double* scal, double* hist_f, double* hist_r, int k, hipStream_t st) {
  hipLaunchKernelGGL(record_kernel, dim3(1), dim3(64), 0, st, scal, hist_f, hist_r, k);
}

void launch_diag(const double* A, int64_t lda, int64_t n, double* sdiag, double* neg,
                 hipStream_t st) {
  hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, A, lda, n, sdiag, neg);
}

template <typename T>
void launch_add(const T* X, const T* Y, T* D, uint16_t* Db, int64_t ld, int64_t n, hipStream_t st) {
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)n);
  hipLaunchKernelGGL(add_kernel<T>, grid, dim3(kThreads), 0, st, X, Y, D, Db, ld, n);
}
template void launch_add<double>(const double*, const double*, double*, uint16_t*, int64_t, int64_t,
                                 hipStream_t);
template void launch_add<float>(const float*, const float*, float*, uint16_t*, int64_t, int64_t,
                                hipStream_t);

template <typename S, typename D>
void launch_convert(const S* src, int64_t lds, int64_t n, D* dst, int64_t ldd, hipStream_t st) {
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)n);
  hipLaunchKernelGGL((convert_kernel<S, D>), grid, dim3(kThreads), 0, st, src, lds, n, dst, ldd);
}
template void launch_convert<double, float>(const double*, int64_t, int64_t, float*, int64_t,
                                            hipStream_t);
template void launch_convert<float, double>(const float*, int64_t, int64_t, double*, int64_t,
                                            hipStream_t);

int64_t launch_gemv_resid(const double* A, int64_t lda, int64_t n, const double* b,
                          const double* theta, double* r, double* partial, hipStream_t st) {
  const int64_t nb = gemv_partials(n);
  hipLaunchKernelGGL(gemv_resid_kernel, dim3((unsigned)nb), dim3(kThreads), 0, st, A, lda, n, b,
                     theta, r, partial, pair_aligned(A, lda, theta) ? 1 : 0);
  return nb;
}

template <typename T>
void launch_gemv_update(const T* G, int64_t ldg, int64_t n, const double* r, double* theta,
                        hipStream_t st) {
  hipLaunchKernelGGL(gemv_update_kernel<T>, dim3((unsigned)((n + 3) / 4)), dim3(kThreads), 0, st, G,
                     ldg, n, r, theta, pair_aligned(G, ldg, r) ? 1 : 0);
}
template void launch_gemv_update<double>(const double*, int64_t, int64_t, const double*, double*,
                                         hipStream_t);
template void launch_gemv_update<float>(const float*, int64_t, int64_t, const double*, double*,
                                        hipStream_t);

template <typename T>
void launch_gemv(const T* M, int64_t ldm, int64_t n, const double* x, const double* z, double* y,
                 int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(gemv_kernel<T>, dim3((unsigned)((n + 3) / 4)), dim3(kThreads), 0, st, M, ldm,
                     n, x, z, y, accumulate, pair_aligned(M, ldm, x) ? 1 : 0);
}
template void launch_gemv<double>(const double*, int64_t, int64_t, const double*, const double*,
                                  double*, int, hipStream_t);
template void launch_gemv<float>(const float*, int64_t, int64_t, const double*, const double*,
                                 double*, int, hipStream_t);

void launch_vec_scale(const double* b, const double* alpha, const double* sdiag, double* theta,
                      int64_t n, int accumulate, hipStream_t st) {
  hipLaunchKernelGGL(vec_scale_kernel, dim3((unsigned)((n + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, st, b, alpha, sdiag, theta, n, accumulate);
}

int64_t launch_vec_sumsq(const double* v, int64_t n, double* partial, hipStream_t st) {
  int64_t nb = (n + kThreads - 1) / kThreads;
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(vec_sumsq_kernel, dim3((unsigned)nb), dim3(kThreads), 0, st, v, n, partial);
  return nb;
}

}  // namespace nsr
