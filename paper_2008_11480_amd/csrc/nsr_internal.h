// Internal declarations shared by the kernels and the solver runtime of libnsr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace nsr {

// D = diag * I + scale * (X Y) + E1 + E2 for row-major float64 operands.
struct GemmF64Args {
  const double* X;
  const double* Y;
  double* D;
  const double* E1;  // may be null
  const double* E2;  // may be null
  int64_t ldx, ldy, ldd, lde1, lde2;
  int64_t M, N, K;
  double diag;
  double scale;
  double* partial;   // per-tile sum of D^2 (null: not wanted)
  int sym;           // 1: symmetric output (M == N): only tiles on or above the
                     // diagonal are computed, the lower triangle is their mirror
  double* sk;        // scratch for split-K tail tiles (may be null: no split)
  int64_t sk_cap;    // its capacity in doubles
  const double* msc; // symmetric output only: null for an exactly symmetric D;
                     // else D[j][i] = D[i][j] msc[j] / msc[i] (D = S^(1/2) D_s
                     // S^(-1/2) with D_s symmetric, S = diag(msc))
};

// D = diag * I + scale * (X op(Y)) + E1 + E2 with float32 output (and an
// optional bf16 copy Db, raw bits), float32 addends.  X / Y are float32 for
// the NN kernel, bf16 (raw 16-bit) for the NT kernel.
struct GemmLpArgs {
  const void* X;
  const void* Y;
  float* D;          // may be null when only Db is wanted
  uint16_t* Db;      // may be null
  const float* E1;   // may be null
  const float* E2;   // may be null
  int64_t ldx, ldy, ldd, lddb, lde1, lde2;
  int64_t M, N, K;
  float diag;
  float scale;
  double* partial;   // per-tile sum of D^2 (float64), may be null
  // Split half-precision NT kernel only: X / Y above are the high planes,
  // Xl / Yl the low planes (same leading dimensions), and xexp[0] / yexp[0]
  // the power-of-two exponents the operands were scaled by.
  const void* Xl;
  const void* Yl;
  const float* xexp;
  const float* yexp;
};

int64_t gemm_lp_partials(int64_t m, int64_t n);
int64_t launch_gemm_f32_nn(const GemmLpArgs& a, hipStream_t st);
int64_t launch_gemm_bf16_nt(const GemmLpArgs& a, hipStream_t st);

// Split float32 operands for the half-precision NT kernel.  absmax writes
// per-block maxima of |X| (returns their count, at most kSplitMaxParts);
// split reads them, picks the exponent e that brings max |X| 2^e into
// [2^14, 2^15), writes e to exp_out[0] and the planes hi = half(X 2^e),
// lo = half(X 2^e - hi): rows x cols row-major (trans = false) or the
// transpose, cols x rows (trans = true), leading dimension ldh (a multiple
// of 8).
constexpr int kSplitMaxParts = 1024;
int64_t launch_absmax(const float* X, int64_t ld, int64_t rows, int64_t cols, float* part,
                      hipStream_t st);
void launch_split_f16(const float* X, int64_t ld, int64_t rows, int64_t cols, const float* part,
                      int64_t nparts, bool trans, uint16_t* hi, uint16_t* lo, int64_t ldh,
                      float* exp_out, hipStream_t st);
// D = diag I + scale (X Y^T) + E1 + E2 from split planes (X: m x k,
// Y: n x k, K contiguous): three half-precision MFMA products
// hi hi + hi lo + lo hi, float32 accumulation, times 2^-(ex + ey).
int64_t launch_gemm_f16s_nt(const GemmLpArgs& a, hipStream_t st);

// Compute units of the current device (queried once).
int device_cus();

// Symmetric-output bf16 NT product (X Y^T symmetric in exact arithmetic,
// m == n): only the upper tiles are computed, the rest is their mirror.
// scratch_floats: what the launch needs for this shape (0 if none, or if the
// shape is better served by the full-output kernel); launch returns the
// number of partials written, -1 on a launch error, -2 if the shape is not
// handled (m != n, or the full-output kernel is faster) or the scratch is too
// small.
int64_t gemm_bf16_sym_scratch_floats(int64_t n, int64_t k);
int64_t launch_gemm_bf16_sym(const GemmLpArgs& a, float* scratch, int64_t scratch_floats,
                             hipStream_t st);

// Upper bound on the number of partials the float64 GEMM writes for an m x n
// output (the size the partial buffer must have).
int64_t gemm_f64_partials(int64_t m, int64_t n, bool sym);

// Scratch (bytes) that lets the float64 GEMM of an m x n x k product split
// the K range of its last, partial round of tiles (0: no split is planned).
size_t gemm_f64_split_bytes(int64_t m, int64_t n, int64_t k, bool sym);

// Enqueue the GEMM; returns the number of partials written (0 if partial is
// null) or a negative value on a launch error.
int64_t launch_gemm_f64(const GemmF64Args& a, hipStream_t st);

// Partial sums of squares of an n x n matrix (one per block); returns the
// number of partials.
int64_t launch_sumsq(const double* A, int64_t lda, int64_t n, double* partial, hipStream_t st);
int64_t sumsq_partials(int64_t n);

// Row sums of |A| -> rowsum (n entries).
void launch_rowabs(const double* A, int64_t lda, int64_t n, double* rowsum, hipStream_t st);

// out[0] = reduce(partial[0..count)) in a fixed order.  mode 0: sum,
// 1: max, 2: sqrt(sum), 3: max / 2 + half_plus_eps.

void launch_reduce(const double* partial, int64_t count, double* out, int mode,
                   double half_plus_eps, hipStream_t st);

// F = I - A S^-1 with S = alpha I (alpha read from device memory) or, when
// sdiag is not null, S = diag(sdiag); computed in float64 and stored as T
// (Fb: optional bf16 copy with the same leading dimension), partial sums of
// F^2.
template <typename T>
int64_t launch_init_resid(const double* A, int64_t lda, int64_t n, const double* alpha,
                          const double* sdiag, T* F, int64_t ldf, uint16_t* Fb, double* partial,
                          hipStream_t st);

// G = S^-1 (I + C) (S as above); C may be null (G = S^-1).
template <typename T>
void launch_scaled_identity_plus(const T* C, int64_t ldc, int64_t n, const double* alpha,
                                 const double* sdiag, T* G, int64_t ldg, hipStream_t st);

// hist_f[k] = scal[1], hist_r[k - 1] = scal[2] (one thread).
void launch_record(const double* scal, double* hist_f, double* hist_r, int k, hipStream_t st);

// sdiag[i] = A_ii, neg[i] = -A_ii.
void launch_diag(const double* A, int64_t lda, int64_t n, double* sdiag, double* neg,
                 hipStream_t st);

// D = X + Y for n x n matrices with leading dimension ld (D may alias X or
// Y); Db: optional bf16 copy of D.
template <typename T>
void launch_add(const T* X, const T* Y, T* D, uint16_t* Db, int64_t ld, int64_t n, hipStream_t st);

// dst = (D) src for an n x n matrix (double <-> float).
template <typename S, typename D>
void launch_convert(const S* src, int64_t lds, int64_t n, D* dst, int64_t ldd, hipStream_t st);

// r = b - A theta, partial sums of r^2 (one per block); returns count.
int64_t launch_gemv_resid(const double* A, int64_t lda, int64_t n, const double* b,
                          const double* theta, double* r, double* partial, hipStream_t st);
int64_t gemv_partials(int64_t n);

// theta += G r (G float64 or float32; float64 accumulation)
template <typename T>
void launch_gemv_update(const T* G, int64_t ldg, int64_t n, const double* r, double* theta,
                        hipStream_t st);

// y = M x + z (z may be null); with accumulate y += M x + z.  M float64 or
// float32, vectors float64.
template <typename T>
void launch_gemv(const T* M, int64_t ldm, int64_t n, const double* x, const double* z, double* y,
                 int accumulate, hipStream_t st);

// theta = S^-1 b (S = alpha I, or diag(sdiag) when sdiag is not null);
// with accumulate theta += S^-1 b.
void launch_vec_scale(const double* b, const double* alpha, const double* sdiag, double* theta,
                      int64_t n, int accumulate, hipStream_t st);

// Sum of squares of a vector -> partials
int64_t launch_vec_sumsq(const double* v, int64_t n, double* partial, hipStream_t st);

// Set the calling thread's ns_last_error() message.
void ns_set_error(const char* msg);

// GEMM families of the tile table (the values of NS_TILE_* in nsr.h).
constexpr int kTileF64 = 0, kTileF32 = 1, kTileBf16 = 2, kTileF16s = 3, kTileFamilies = 4;
// Tile edge set by the tile autotuner for an m x n output of a family, or 0
// (use the library's rule).
int tile_choice(int family, int64_t m, int64_t n);


// ---------------------------------------------------------------------------
// LDS DMA (device code of the GEMMs that stage operands with
// global_load_lds_dwordx4).
// ---------------------------------------------------------------------------
// One LDS DMA instruction: 16 bytes per lane from src to LDS byte address
// lds + 16 * lane (lds wave-uniform).  Written as inline assembly so that
// the compiler, which does not see these LDS writes, adds no wait of its own
// before the operand reads: the kernels order them themselves (vmcnt +
// barrier).  m0 is set right before the load (one wait state between the
// two); no other code of these kernels uses m0.
__device__ __forceinline__ void lds_dma16(const void* src, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(src), "s"(lds)
               : "memory");
}

// The same with a wave-uniform base address and a 32-bit per-lane byte offset
// (one VGPR per instruction instead of a pair).
__device__ __forceinline__ void lds_dma16s(const void* base, uint32_t off, uint32_t lds) {
  asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
               :
               : "v"(off), "s"(base), "s"(lds)
               : "memory");
}

// Wait until at most CNT of this wave's DMA instructions are outstanding and
// its LDS reads are complete, then the workgroup barrier.
template <int CNT>
__device__ __forceinline__ void dma_wait_barrier() {
  asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" : : "n"(CNT) : "memory");
}

// fn(std::integral_constant<int, I>) for I = B .. E - 1, unrolled at compile
// time (a loop the compiler only partly unrolls would index register arrays
// at run time, which puts them in scratch).
template <int B, int E, typename Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  if constexpr (B < E) {
    fn(std::integral_constant<int, B>{});
    static_for<B + 1, E>(fn);
  }
}

// LDS byte address of a shared-memory object (the low 32 bits of its
// generic address).
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return (uint32_t)reinterpret_cast<uintptr_t>(p);
}

}  // namespace nsr
