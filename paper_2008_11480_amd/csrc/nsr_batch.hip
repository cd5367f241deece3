// Batched solves of many independent SPD systems of uneven size in one
// persistent launch per precision.
//
// Each workgroup pulls whole systems from a device counter (systems are
// pre-sorted by decreasing n, so the largest start first) and runs the
// complete coupled solve of one system inside the workgroup: the scalar
// preconditioner (Section 2), Newton-Schulz steps of order 2^s in the
// factorized form (I+F)(I+F^2)... (eq. ns, Tables 1-2), the coupled
// Richardson update (eq. redttk1), the stop rule and float64 refinement.  The
// float32 pass runs the products in float32 MFMA (v_mfma_f32_16x16x4_f32) and
// queues the systems it cannot bring to the tolerance; a second kernel
// re-solves those in float64 MFMA (v_mfma_f64_16x16x4_f64).  Workgroups never
// wait for each other: a workgroup exits when the counter has passed the
// number of systems.
//
// General kernel: matrices live in the workgroup's slot of the workspace
// (row-major, leading dimension ldw); products walk the output in blocks
// staged through LDS (wg_gemm).  Submissions whose systems all have
// n <= SMALL_N (orders 2 and 4) run a second kernel that keeps the whole
// iteration in LDS (wg_solve_small).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "nsr.h"
#include "nsr_internal.h"

// K slab of the in-workgroup GEMM (elements), float32 and float64 (eight-wave
// workgroups).
#ifndef NSR_BATCH_KB32
#define NSR_BATCH_KB32 16
#endif
#ifndef NSR_BATCH_KB64
#define NSR_BATCH_KB64 16
#endif
// Rows of the residual / update GEMVs whose loads are issued together (2
// measured best on the 2048-system harmonic batch: 3 and more cost the float32
// pass registers, 1 leaves loads of one row in flight at a time).
#ifndef NSR_BATCH_GR
#define NSR_BATCH_GR 2
#endif
// 1: float32 in-workgroup products stage their K slabs by LDS DMA.
#ifndef NSR_BATCH_F32_DMA
#define NSR_BATCH_F32_DMA 1
#endif
// 1: float64 re-solves of escalated systems run in lockstep across the GPU
// (batches of at least kLsMinCount systems whose largest has n >= kLsMinN).
#ifndef NSR_BATCH_LOCKSTEP
#define NSR_BATCH_LOCKSTEP 1
#endif

namespace nsr {

struct BatchDesc {
  const double* A;
  const double* b;
  double* theta;
  int64_t lda;
  int32_t n;
  int32_t pad;
};

struct BatchResult {
  int32_t status, ns_stop, refine_stop, ns_steps, refine_steps, precision, n_fnorm, n_resid;
  double alpha, rel_resid;
  int64_t mmm;
  int64_t clock[4];    // wall-clock ticks: float32 attempt begin / end, float64 begin / end
  int32_t wg[2];       // workgroup of each attempt (-1: not run)
  double fnorm_hist[NS_HIST_F];
};

struct BatchArgs {
  const BatchDesc* desc;
  BatchResult* res;
  const int32_t* order;   // processing order (indices into desc)
  int32_t* counter;       // kCounters, zeroed before launch: [0] float32 /
                          // float64-only work counter, [1] float64 queue entries
                          // claimed, [2] queue length, [3] float64 re-solves
                          // finished, [4] float32 attempts finished, [5] error
                          // flag of a timed-out wait (escalating kernel),
                          // [6] overflow entries claimed, [7] overflow length
  int32_t* retry;         // queue of systems for float64 (count entries; an
                          // entry holds sid + 1 once written, 0 before)
  struct TeamState* team; // per queue entry: its float64 team (escalating kernel)
  char* slots;
  int64_t slot_bytes;
  int32_t count;
  int32_t ldw;            // slot leading dimension (>= max n, multiple of 4)
  int32_t ns_order;       // 2^s
  int32_t k_max;
  int32_t refine_max;
  int32_t floor_detect;
  int32_t escalate;       // 1: float32 first, float64 when it fails
  int32_t fp64_only;      // 1: float64 from the start
  int32_t scale;           // ns_scale
  int32_t slot_base;       // first slot of this launch (the team kernel's follow
                           // the float32 pass's)
  int32_t ls_on;           // 1: the queue is re-solved in lockstep; the float64
                           // pass then takes the overflow queue
  int32_t ls_slots;        // slots the lockstep re-solve may use (queue entry q
                           // uses slot q)
  struct LsState* ls;      // per queue entry: lockstep state
  int32_t* ovf;            // overflow queue (sid + 1): entries beyond the slots,
                           // systems still iterating after the enqueued steps
  int64_t ticks_ms;        // device wall-clock ticks per millisecond
  double eps;              // NS_SCALE_INF_HALF: alpha = ||A||_inf / 2 + eps
  double f_tol;
  double resid_tol;
};

// Products of one float64 re-solve shared block by block with idle
// workgroups (the escalating kernel).  The leader publishes each product
// ("phase") here; any workgroup may claim a block of the current phase by a
// compare-and-swap on `claim`, and adds 1 to `done` when the block is
// written.  Zeroed before launch.
struct TeamDesc {
  const double* X;
  const double* XA;
  const double* Y;
  double* D;
  const double* E1;
  const double* E2;
  double* part;       // per-block sums of D^2 (the leader's slot)
  int64_t lda;
  double diag, scale;
  int32_t n, ldx, ldy, ldd, lde, total, want_ss;
  uint32_t seq;       // phase number (1, 2, ...)
};
struct TeamState {
  unsigned long long claim;   // (phase << 32) | next unclaimed block
  int32_t done;               // blocks finished in the current phase
  int32_t active;             // 1 while the leader runs
  TeamDesc desc;
};

// State of one system's lockstep float64 re-solve (see the lockstep kernels).
struct LsState {
  double alpha, f0, fprev, fk, bnorm;
  int64_t mmm;       // float64 products (write_result adds the float32 attempt's)
  int64_t t_begin;
  int32_t sid, n, k, ns_stop, active, implicit, gc, f2_ready, probe, pad;
};

constexpr int kCounters = 8;

namespace {

// Margin of the error-law floor test of the stop rule.
constexpr double kLawMargin = 1e3;
// Bounds of the team kernel's waits, in milliseconds of the device wall
// clock: a wait for work another workgroup holds (a claimed block, a queue
// entry being written) sets the error flag and ends after kWaitMs; a team
// workgroup with nothing to do exits after kIdleMs without work, or after
// kStartMs if the float32 pass has not started beside it.
constexpr int64_t kWaitMs = 2000, kIdleMs = 200, kStartMs = 2;

// Polls use relaxed agent-scope atomic loads, which read the coherent value
// without cache maintenance; the acquire fence (an L2 invalidate on this
// chip) is issued once, after the awaited value is seen, and producers
// issue a release fence (an L2 write-back) before publishing.  An acquire
// load in a spin loop would invalidate the L2 of the whole XCD on every
// iteration, under every other workgroup's products.
__device__ __forceinline__ int ld_rlx(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_rlx64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ __forceinline__ void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the workgroup, same value returned to every thread.
template <int NW>
__device__ __forceinline__ double block_sum_all(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wsum(v);
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Maximum over the workgroup, same value returned to every thread.
template <int NW>
__device__ __forceinline__ double block_max_all(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double m = red[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) m = fmax(m, red[w]);
  __syncthreads();
  return m;
}

__device__ __forceinline__ f32x4 mfma(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc;
template <> struct Acc<float> { typedef f32x4 type; };
template <> struct Acc<double> { typedef f64x4 type; };

// Row of accumulator element r of lane group lk (lane / 16) in a 16x16 block:
// float32: 4 lk + r; float64: lk + 4 r (gfx950 layouts).
__device__ __forceinline__ int acc_row(float, int lk, int r) { return 4 * lk + r; }
__device__ __forceinline__ int acc_row(double, int lk, int r) { return lk + 4 * r; }

// In-workgroup GEMM tiling: the n x n output is walked in BM x BN blocks
// (32 x 32 for one wave, 64 x 32 for two, 64 x 64 for four, 128 x 64 for
// eight), one 32 x 32 sub-block (2 x 2 MFMA blocks of 16 x 16) per wave.
// The K range of a block is walked in slabs of KB (16 float32; 16 float64 on
// eight waves, else 8)
// staged global -> registers (one slab ahead, 16-byte loads) -> two LDS
// buffers -> MFMA fragments, one barrier per slab.
template <int NW> struct Block {
  static constexpr int BM = NW >= 8 ? 128 : (NW >= 2 ? 64 : 32);
  static constexpr int BN = NW >= 4 ? 64 : 32;
  static_assert((BM / 32) * (BN / 32) == NW, "one 32 x 32 sub-block per wave");
};
template <typename T, int NW> struct Stage {
  // K slab: the float64 slab of 16 pays on the eight-wave workgroups of the
  // float64 pass; narrower workgroups keep 8 (their registers spill with 16).
  static constexpr int KB = sizeof(T) == 4 ? NSR_BATCH_KB32 : (NW >= 8 ? NSR_BATCH_KB64 : 8);
  static constexpr int VE = 16 / (int)sizeof(T);       // elements per 16-byte load
  static constexpr int XS = KB + (sizeof(T) == 4 ? 4 : 2);
  static constexpr int YS = Block<NW>::BN + (sizeof(T) == 4 ? 4 : 2);
  static constexpr int BUF = Block<NW>::BM * XS + KB * YS;   // one buffer, elements
  static constexpr int BYTES = 2 * BUF * (int)sizeof(T);
};

typedef float f32v4 __attribute__((ext_vector_type(4)));
typedef double f64v2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { typedef f32v4 type; };
template <> struct Vec16<double> { typedef f64v2 type; };

// Output blocks of an n x n product (Block<NW> tiling).
template <typename T, int NW>
__device__ __forceinline__ int wg_gemm_blocks(int n) {
  return ((n + Block<NW>::BM - 1) / Block<NW>::BM) * ((n + Block<NW>::BN - 1) / Block<NW>::BN);
}

// One BM x BN output block (index blk in row-major block order) of
// D = diag I + scale X Y + E1 + E2; returns this thread's share of the
// block's sum D^2 (not reduced).  All threads call it; it ends with a
// barrier.
template <typename T, int NW>
__device__ double wg_gemm_block(int blk, int n, const T* X, int ldx, const double* XA,
                                int64_t lda, const T* Y, int ldy, T* D, int ldd, const T* E1,
                                const T* E2, int lde, T diag, T scale, void* lds) {
  typedef typename Acc<T>::type acc_t;
  typedef typename Vec16<T>::type vec_t;
  typedef Stage<T, NW> S;
  constexpr int KB = S::KB, VE = S::VE, XS = S::XS, YS = S::YS;
  constexpr int BM = Block<NW>::BM, BN = Block<NW>::BN;
  constexpr int NTH = NW * 64;
  constexpr int XV = KB / VE, YV = BN / VE;      // 16-byte vectors per slab row
  constexpr int XTOT = BM * XV, YTOT = KB * YV;  // vectors per slab
  constexpr int XPER = (XTOT + NTH - 1) / NTH, YPER = (YTOT + NTH - 1) / NTH;
  // Keep the per-thread index arithmetic inside each call: the solver calls
  // this from several places in one loop, and hoisting every call's
  // invariants out of that loop would exhaust the register file.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  T* Xs[2] = {reinterpret_cast<T*>(lds), reinterpret_cast<T*>(lds) + S::BUF};
  T* Ys[2] = {Xs[0] + BM * XS, Xs[1] + BM * XS};
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int sr = (wave / (BN / 32)) * 32, sc = (wave % (BN / 32)) * 32;
  const bool xa_vec = XA && ((lda & 1) == 0) && ((reinterpret_cast<uintptr_t>(XA) & 15) == 0);
  const int nbn = (n + BN - 1) / BN;
  const int nk = (n + KB - 1) / KB;
  double ss = 0.0;
  {
    const int r0 = (blk / nbn) * BM, c0 = (blk % nbn) * BN;
    const bool active = (r0 + sr < n) && (c0 + sc < n);   // wave-uniform
    vec_t xr[XPER], yr[YPER];
    auto load = [&](int k0) {
#pragma unroll
      for (int u = 0; u < XPER; ++u) {
        const int v = tid + NTH * u;
        const int row = r0 + v / XV, col = k0 + (v % XV) * VE;
        vec_t val;
#pragma unroll
        for (int e = 0; e < VE; ++e) val[e] = T(0);
        if (v < XTOT && row < n) {
          if (XA) {
            const double* src = XA + (int64_t)row * lda + col;
            if (sizeof(T) == 8 && xa_vec && col + VE <= n) {
              val = *reinterpret_cast<const vec_t*>(src);
            } else {
#pragma unroll
              for (int e = 0; e < VE; ++e)
                if (col + e < n) val[e] = (T)src[e];
            }
          } else {
            const T* src = X + row * ldx + col;
            if (col + VE <= n) {
              val = *reinterpret_cast<const vec_t*>(src);
            } else {
#pragma unroll
              for (int e = 0; e < VE; ++e)
                if (col + e < n) val[e] = src[e];
            }
          }
        }
        xr[u] = val;
      }
#pragma unroll
      for (int u = 0; u < YPER; ++u) {
        const int v = tid + NTH * u;
        const int row = k0 + v / YV, col = c0 + (v % YV) * VE;
        vec_t val;
#pragma unroll
        for (int e = 0; e < VE; ++e) val[e] = T(0);
        if (v < YTOT && row < n) {
          const T* src = Y + row * ldy + col;
          if (col + VE <= n) {
            val = *reinterpret_cast<const vec_t*>(src);
          } else {
#pragma unroll
            for (int e = 0; e < VE; ++e)
              if (col + e < n) val[e] = src[e];
          }
        }
        yr[u] = val;
      }
    };
    auto store = [&](T* xs, T* ys) {
#pragma unroll
      for (int u = 0; u < XPER; ++u) {
        const int v = tid + NTH * u;
        if (v < XTOT) *reinterpret_cast<vec_t*>(&xs[(v / XV) * XS + (v % XV) * VE]) = xr[u];
      }
#pragma unroll
      for (int u = 0; u < YPER; ++u) {
        const int v = tid + NTH * u;
        if (v < YTOT) *reinterpret_cast<vec_t*>(&ys[(v / YV) * YS + (v % YV) * VE]) = yr[u];
      }
    };
    acc_t acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = acc_t{0, 0, 0, 0};
    load(0);
    for (int kt = 0; kt < nk; ++kt) {
      T* xsb = (kt & 1) ? Xs[1] : Xs[0];
      T* ysb = (kt & 1) ? Ys[1] : Ys[0];
      store(xsb, ysb);
      __syncthreads();
      if (kt + 1 < nk) load((kt + 1) * KB);
      if (active) {
        const T* xs = xsb + (sr + lr) * XS + lk;
        const T* ys = ysb + lk * YS + sc + lr;
#pragma unroll
        for (int ks = 0; ks < KB; ks += 4) {
          const T a0 = xs[ks], a1 = xs[16 * XS + ks];
          const T b0 = ys[ks * YS], b1 = ys[ks * YS + 16];
          acc[0][0] = mfma(a0, b0, acc[0][0]);
          acc[0][1] = mfma(a0, b1, acc[0][1]);
          acc[1][0] = mfma(a1, b0, acc[1][0]);
          acc[1][1] = mfma(a1, b1, acc[1][1]);
        }
      }
    }
    if (active) {
      // The addends of a row of fragments are loaded before its stores:
      // loads and stores share one in-order completion counter, so a load
      // issued after a store waits for that store.
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        T e1[2][4], e2[2][4];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = c0 + sc + 16 * j + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + sr + 16 * i + acc_row(T(0), lk, r);
            const bool in = row < n && col < n;
            e1[j][r] = (E1 && in) ? E1[row * lde + col] : T(0);
            e2[j][r] = (E2 && in) ? E2[row * lde + col] : T(0);
          }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = c0 + sc + 16 * j + lr;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = r0 + sr + 16 * i + acc_row(T(0), lk, r);
            if (row < n && col < n) {
              T v = scale * acc[i][j][r];
              if (row == col) v += diag;
              if (E1) v += e1[j][r];
              if (E2) v += e2[j][r];
              D[row * ldd + col] = v;
              ss += (double)v * (double)v;
            }
          }
        }
      }
    }
    __syncthreads();  // LDS buffers free for the next block, D complete
  }
  return ss;
}

// ---------------------------------------------------------------------------
// Float32 products fed by LDS DMA.  Operands are slot matrices (leading
// dimension ldw, a multiple of 32) whose rows and columns n .. ceil32(n) - 1
// are zero (wg_zero_pads), so K runs in whole 32-deep slabs.  Each slab goes
// from global memory straight into a ring of three LDS stages, two slabs
// ahead of the MFMAs; one barrier per slab.  Rows of X past n (and columns
// of Y past ldw) read row n - 1 (column ldw - 4) instead: they only feed
// outputs that are not stored.
//
// LDS: X rows of 32 floats (8 chunks of 16 bytes, chunk c stored at c ^
// ((row >> 1) & 7)), then 32 Y rows of BN floats (chunk c at c ^ ysw(k)).
// An operand read of the 16 x 16 x 4 MFMA (16 rows or columns, 4 k) then
// touches 64 different banks.
// ---------------------------------------------------------------------------
template <int NW> struct DmaF32 {
  static constexpr int BM = Block<NW>::BM, BN = Block<NW>::BN, KB = 32, NST = 3;
  static constexpr int XBYTES = BM * KB * 4, YBYTES = KB * BN * 4;
  static constexpr int SBYTES = XBYTES + YBYTES, BYTES = NST * SBYTES;
  static constexpr int YCH = BN / 4;            // 16-byte chunks per Y row
  static constexpr int YR = 64 / YCH;           // Y rows per DMA instruction
  static constexpr int XI = (BM / 8) / NW;      // DMA instructions per wave and slab
  static constexpr int YI = (KB / YR) / NW;
  static constexpr int PER = XI + YI;
  static_assert(XI * NW * 8 == BM && YI * NW * YR == KB, "DMA split");
};
// Y chunk permutation for k row kr: rows of one 256-byte bank window are
// separated by their 128-byte half, rows of the four k of an MFMA step by
// the chunk group.
template <int YCH>
__device__ __forceinline__ int dma_ysw(int kr) {
  return YCH >= 16 ? 4 * (kr & 3) : 4 * ((kr >> 1) & 1);
}

// LDS bytes of a workgroup's GEMM stages.
template <typename T, int NW> struct StageBytes {
  static constexpr int value =
      (sizeof(T) == 4 && NSR_BATCH_F32_DMA) ? DmaF32<NW>::BYTES : Stage<T, NW>::BYTES;
};

// Zero rows and columns n .. ceil32(n) - 1 (within the first ceil32(n) rows
// and columns) of the eight float32 slot matrices starting at m0 (ldw^2
// floats apart).
template <int NW>
__device__ void wg_zero_pads(int n, float* m0, int ldw) {
  const int kp = (n + 31) & ~31;
  const int w = kp - n;   // pad width
  if (w == 0) return;
  const int per = 2 * n * w + w * w;   // [0,n) x [n,kp), [n,kp) x [0,kp)
  for (int mtx = 0; mtx < 8; ++mtx) {
    float* M = m0 + (int64_t)mtx * ldw * ldw;
    for (int e = threadIdx.x; e < per; e += NW * 64) {
      int row, col;
      if (e < n * w) {
        row = e / w;
        col = n + e % w;
      } else {
        const int f = e - n * w;
        row = n + f / kp;
        col = f % kp;
      }
      M[row * ldw + col] = 0.0f;
    }
  }
  __syncthreads();
}

template <int NW>
__device__ double wg_gemm_block_dma(int blk, int n, const float* X, const float* Y, float* D,
                                    int ldw, const float* E1, const float* E2, float diag,
                                    float scale, void* lds) {
  typedef DmaF32<NW> S;
  constexpr int BM = S::BM, BN = S::BN, KB = S::KB, NST = S::NST, YCH = S::YCH;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nbn = (n + BN - 1) / BN;
  const int r0 = (blk / nbn) * BM, c0 = (blk % nbn) * BN;
  const int nk = (n + KB - 1) / KB;
  unsigned char* ring = static_cast<unsigned char*>(lds);
  const uint32_t ring_lds = lds_addr(ring);
  // DMA sources (k offset added per slab)
  const float* xs[S::XI];
  const float* ys[S::YI];
#pragma unroll
  for (int u = 0; u < S::XI; ++u) {
    const int r = (u * NW + wave) * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    const int gr = r0 + r < n ? r0 + r : n - 1;
    xs[u] = X + (int64_t)gr * ldw + 4 * c;
  }
#pragma unroll
  for (int u = 0; u < S::YI; ++u) {
    const int kr = (u * NW + wave) * S::YR + lane / YCH;
    const int c = (lane % YCH) ^ dma_ysw<YCH>(kr);
    int col = c0 + 4 * c;
    if (col > ldw - 4) col = ldw - 4;
    ys[u] = Y + (int64_t)kr * ldw + col;
  }
  auto issue = [&](int kt) {
    const uint32_t st = ring_lds + (uint32_t)((kt % NST) * S::SBYTES);
    const int64_t k0 = (int64_t)kt * KB;
#pragma unroll
    for (int u = 0; u < S::XI; ++u)
      lds_dma16(xs[u] + k0, st + (uint32_t)((u * NW + wave) * 8 * KB * 4));
#pragma unroll
    for (int u = 0; u < S::YI; ++u)
      lds_dma16(ys[u] + k0 * ldw, st + (uint32_t)(S::XBYTES + (u * NW + wave) * 1024));
  };
  const int lr = lane & 15, lk = lane >> 4;
  const int sr = (wave / (BN / 32)) * 32, sc = (wave % (BN / 32)) * 32;
  const bool active = (r0 + sr < n) && (c0 + sc < n);   // wave-uniform
  const int xsw = (lr >> 1) & 7;                        // row swizzle of this lane's rows
  const int ysw = dma_ysw<YCH>(lk);                     // k row swizzle (k = ks + lk, ks % 4 == 0)
  const int offa = (sr + lr) * KB * 4 + 4 * lk;
  int offb[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
    offb[j] = S::XBYTES + lk * BN * 4 + 16 * (((sc + 16 * j + lr) >> 2) ^ ysw) + 4 * (lr & 3);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
  issue(0);
  if (nk > 1) issue(1);
  for (int kt = 0; kt < nk; ++kt) {
    const int later = nk - 1 - kt;
    if (later >= 1)
      dma_wait_barrier<S::PER>();
    else
      dma_wait_barrier<0>();
    if (kt + 2 < nk) issue(kt + 2);
    if (active) {
      const unsigned char* st = ring + (kt % NST) * S::SBYTES;
#pragma unroll
      for (int ks = 0; ks < KB; ks += 4) {
        const int ca = 16 * ((ks >> 2) ^ xsw);
        const float a0 = *reinterpret_cast<const float*>(st + offa + ca);
        const float a1 = *reinterpret_cast<const float*>(st + offa + 16 * KB * 4 + ca);
        const float b0 = *reinterpret_cast<const float*>(st + offb[0] + ks * BN * 4);
        const float b1 = *reinterpret_cast<const float*>(st + offb[1] + ks * BN * 4);
        acc[0][0] = mfma(a0, b0, acc[0][0]);
        acc[0][1] = mfma(a0, b1, acc[0][1]);
        acc[1][0] = mfma(a1, b0, acc[1][0]);
        acc[1][1] = mfma(a1, b1, acc[1][1]);
      }
    }
  }
  double ss = 0.0;
  if (active) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      float e1[2][4], e2[2][4];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = c0 + sc + 16 * j + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + sr + 16 * i + acc_row(0.0f, lk, r);
          const bool in = row < n && col < n;
          e1[j][r] = (E1 && in) ? E1[row * ldw + col] : 0.0f;
          e2[j][r] = (E2 && in) ? E2[row * ldw + col] : 0.0f;
        }
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = c0 + sc + 16 * j + lr;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = r0 + sr + 16 * i + acc_row(0.0f, lk, r);
          if (row < n && col < n) {
            float v = scale * acc[i][j][r];
            if (row == col) v += diag;
            if (E1) v += e1[j][r];
            if (E2) v += e2[j][r];
            D[row * ldw + col] = v;
            ss += (double)v * (double)v;
          }
        }
      }
    }
  }
  __syncthreads();  // the ring is free for the next block, D complete
  return ss;
}

// D = diag I + scale X Y + E1 + E2 (n x n); returns sum D^2 over the
// workgroup when want_ss (uniform).  XA: X is the float64 input A (read
// through lda), otherwise X is T with leading dimension ldx (multiple of 4).
// lds: Stage<T, NW>::BYTES of LDS shared by the workgroup.
template <typename T, int NW>
__device__ double wg_gemm(int n, const T* X, int ldx, const double* XA, int64_t lda, const T* Y,
                          int ldy, T* D, int ldd, const T* E1, const T* E2, int lde, T diag,
                          T scale, bool want_ss, double* red, void* lds) {
  double ss = 0.0;
  const int nb = wg_gemm_blocks<T, NW>(n);
  if constexpr (sizeof(T) == 4 && NSR_BATCH_F32_DMA) {
    // float32 operands are always slot matrices (leading dimension ldx ==
    // ldy == ldd == lde, zero pads), never the float64 input
    for (int blk = 0; blk < nb; ++blk)
      ss += wg_gemm_block_dma<NW>(blk, n, (const float*)X, (const float*)Y, (float*)D, ldd,
                                  (const float*)E1, (const float*)E2, (float)diag, (float)scale,
                                  lds);
  } else {
    for (int blk = 0; blk < nb; ++blk)
      ss += wg_gemm_block<T, NW>(blk, n, X, ldx, XA, lda, Y, ldy, D, ldd, E1, E2, lde, diag,
                                 scale, lds);
  }
  if (!want_ss) return 0.0;
  return block_sum_all<NW>(ss, red);
}

// Elementwise passes over the n x n slot matrices, all threads.  Each thread
// loads EW elements before it stores them: loads and stores share one
// in-order completion counter, so a load issued after a store waits for it,
// and one element per iteration would cost a memory round trip each.
constexpr int EW = 8;

template <typename T, int NW>
__device__ double wg_init_resid(int n, const double* A, int64_t lda, double alpha,
                                const double* sd, T* F, int ldw, double* red) {
  constexpr int NTH = NW * 64;
  const int nn = n * n;
  double ss = 0.0;
  for (int i0 = threadIdx.x; i0 < nn; i0 += NTH * EW) {
    double a[EW];
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      a[u] = i < nn ? A[(int64_t)(i / n) * lda + i % n] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      if (i < nn) {
        const int row = i / n, col = i % n;
        double v = -a[u] / (sd ? sd[col] : alpha);   // F_0 = I - A S^-1
        if (row == col) v += 1.0;
        const T t = (T)v;
        F[row * ldw + col] = t;
        ss += (double)t * (double)t;
      }
    }
  }
  __syncthreads();
  return block_sum_all<NW>(ss, red);
}

template <typename T, int NW>
__device__ void wg_scaled_identity_plus(int n, const T* C, double alpha, const double* sd, T* G,
                                        int ldw) {
  constexpr int NTH = NW * 64;
  const int nn = n * n;
  for (int i0 = threadIdx.x; i0 < nn; i0 += NTH * EW) {
    T c[EW];
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      c[u] = i < nn ? C[(i / n) * ldw + i % n] : T(0);
    }
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      if (i < nn) {
        const int row = i / n, col = i % n;
        double v = (double)c[u];
        if (row == col) v += 1.0;
        G[row * ldw + col] = (T)(v / (sd ? sd[row] : alpha));   // G_1 = S^-1 (I + C)
      }
    }
  }
  __syncthreads();
}

// Copy of A in precision T (leading dimension ldw).
template <typename T, int NW>
__device__ void wg_copy_A(int n, const double* A, int64_t lda, T* AT, int ldw) {
  constexpr int NTH = NW * 64;
  const int nn = n * n;
  for (int i0 = threadIdx.x; i0 < nn; i0 += NTH * EW) {
    double a[EW];
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      a[u] = i < nn ? A[(int64_t)(i / n) * lda + i % n] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < EW; ++u) {
      const int i = i0 + u * NTH;
      if (i < nn) AT[(i / n) * ldw + i % n] = (T)a[u];
    }
  }
  __syncthreads();
}

// r = b - A theta (float64), returns ||r||^2 (uniform).  Wave w owns rows
// w, w + NW, ...; it takes them GR at a time, issuing the GR rows' loads
// together, and in each chunk of 64 of its rows lane j keeps row j's value;
// the chunk is stored at once after its loads (loads and stores share one
// in-order completion counter, so storing per row would cost a memory round
// trip per row).  GR trades registers for loads in flight.
template <int NW, int GR>
__device__ double wg_resid(int n, const double* A, int64_t lda, const double* b,
                           const double* theta, double* r, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double ss = 0.0;
  for (int base = wave; base < n; base += 64 * NW) {
    double mine = 0.0;
    int myrow = -1;
    for (int j0 = 0; j0 < 64 && base + j0 * NW < n; j0 += GR) {
      double s[GR];
#pragma unroll
      for (int u = 0; u < GR; ++u) s[u] = 0.0;
      for (int c = lane; c < n; c += 64) {
        const double t = theta[c];
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int row = base + (j0 + u) * NW;
          if (row < n) s[u] += A[(int64_t)row * lda + c] * t;
        }
      }
#pragma unroll
      for (int u = 0; u < GR; ++u) {
        const int row = base + (j0 + u) * NW;
        const double sv = wsum(s[u]);
        if (row < n && lane == j0 + u) {
          mine = b[row] - sv;
          myrow = row;
        }
      }
    }
    if (myrow >= 0) {
      r[myrow] = mine;
      ss += mine * mine;
    }
  }
  __syncthreads();
  return block_sum_all<NW>(ss, red);
}

// theta += G r (G of type T, or G = I / alpha when implicit); rows grouped
// and chunked per wave as in wg_resid.
template <typename T, int NW, int GR>
__device__ void wg_update(int n, const T* G, int ldw, bool implicit, double alpha, const double* r,
                          double* theta) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int base = wave; base < n; base += 64 * NW) {
    double mine = 0.0;
    int myrow = -1;
    for (int j0 = 0; j0 < 64 && base + j0 * NW < n; j0 += GR) {
      double s[GR];
#pragma unroll
      for (int u = 0; u < GR; ++u) s[u] = 0.0;
      if (implicit) {
#pragma unroll
        for (int u = 0; u < GR; ++u) {
          const int row = base + (j0 + u) * NW;
          if (row < n && lane == 0) s[u] = r[row] / alpha;
        }
      } else {
        for (int c = lane; c < n; c += 64) {
          const double rc = r[c];
#pragma unroll
          for (int u = 0; u < GR; ++u) {
            const int row = base + (j0 + u) * NW;
            if (row < n) s[u] += (double)G[row * ldw + c] * rc;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < GR; ++u) {
        const int row = base + (j0 + u) * NW;
        const double sv = wsum(s[u]);
        if (row < n && lane == j0 + u) {
          mine = sv;
          myrow = row;
        }
      }
    }
    if (myrow >= 0) theta[myrow] += mine;
  }
  __syncthreads();
}

struct SlotMats {
  void* G[2];
  void* F;
  void* P[2];
  void* C[2];
  float* A32;
  double* r;
  double* sd;  // S = diag(A) (NS_SCALE_DIAG), n values
  void* lds;   // Stage<T, NW>::BYTES of LDS for the GEMM stages
};

// Control values of one solve.  Every thread holds the same values (they are
// computed from workgroup-wide sums); only thread 0 writes the history.
struct Ctl {
  double alpha, rel_resid;
  int64_t mmm;
  int ns_steps, ns_stop, refine_steps, refine_stop, n_fnorm, precision;
};

// Preconditioner S (Section 2): S = alpha I with alpha = ||A||_F, or the
// maximum row sum of |A| over 2 plus eps; or S = diag(A), written to sd,
// reporting alpha = max_i A_ii (-1 when a diagonal entry is not finite and
// positive).  Uniform result.
template <int NW>
__device__ __forceinline__ double wg_alpha(const BatchArgs& P, const BatchDesc& d, double* red,
                                           double* sd) {
  const int n = d.n;
  if (P.scale == NS_SCALE_DIAG) {
    double mx = 0.0;
    for (int i = threadIdx.x; i < n; i += NW * 64) {
      const double a = d.A[(int64_t)i * d.lda + i];
      sd[i] = a;
      mx = (a > 0.0 && isfinite(a)) ? fmax(mx, a) : INFINITY;
    }
    const double m = block_max_all<NW>(mx, red);   // its barriers publish sd
    return isfinite(m) ? m : -1.0;
  }
  if (P.scale == NS_SCALE_INF_HALF) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double mx = 0.0;
    for (int row = wave; row < n; row += NW) {
      double rs = 0.0;
      for (int col = lane; col < n; col += 64) rs += fabs(d.A[(int64_t)row * d.lda + col]);
      mx = fmax(mx, wsum(rs));
    }
    return 0.5 * block_max_all<NW>(mx, red) + P.eps;
  }
  double ssa = 0.0;
  for (int i = threadIdx.x; i < n * n; i += NW * 64) {
    const double v = d.A[(int64_t)(i / n) * d.lda + (i % n)];
    ssa += v * v;
  }
  return sqrt(block_sum_all<NW>(ssa, red));
}

// theta_0 = S^-1 b; returns ||b|| (1 for b = 0), uniform.
template <int NW>
__device__ __forceinline__ double wg_theta0(int n, const double* b, double* theta, double alpha,
                                            const double* sd, double* red) {
  double bb = 0.0;
  for (int i = threadIdx.x; i < n; i += NW * 64) {
    theta[i] = b[i] / (sd ? sd[i] : alpha);
    bb += b[i] * b[i];
  }
  const double bnorm = sqrt(block_sum_all<NW>(bb, red));
  return bnorm == 0.0 ? 1.0 : bnorm;
}

// Float32 attempt that can escalate: with order^(k32 - 1) >= ln 2 / 2^-24,
// every eigenvalue mu <= 1 - 2^-24 of F_0 has mu^(order^(k32 - 1)) <= 1/2
// (eq. fk1), so at step k32 + 1 it is below 2^-(order^2).  Returns k32 + 1.
__device__ __forceinline__ int bail_step(int order) {
  double e = 1.0;
  int k32 = 1;
  while (e < 0.6931471805599453 * 16777216.0) {
    e *= (double)order;
    ++k32;
  }
  return k32 + 1;
}

// Richardson refinement with the final G (eq. redttk1) until the relative
// residual reaches resid_tol, refine_max steps, or a stall (less than a
// factor 2 over 3 steps).  A (float64, leading dimension lda), b, theta and
// the scratch r hold n values each.  Returns true on resid_tol.
template <typename T, int NW, int GR>
__device__ __forceinline__ bool wg_refine(const BatchArgs& P, int n, const double* A, int64_t lda,
                                          const double* b, double* theta, const T* G, int ldg,
                                          double alpha, double* r, double bnorm, double* red,
                                          Ctl& c) {
  double last[4] = {0, 0, 0, 0};
  int refine = 0;
  while (true) {
    const double rel = sqrt(wg_resid<NW, GR>(n, A, lda, b, theta, r, red)) / bnorm;
    c.rel_resid = rel;
    for (int j = 3; j > 0; --j) last[j] = last[j - 1];
    last[0] = rel;
    if (!isfinite(rel)) {
      c.refine_stop = NS_STOP_DIVERGED;
      break;
    }
    if (rel <= P.resid_tol) {
      c.refine_stop = NS_STOP_RESID_TOL;
      break;
    }
    if (refine >= P.refine_max) {
      c.refine_stop = NS_STOP_REFINE_MAX;
      break;
    }
    if (refine >= 3 && rel > 0.5 * last[3]) {
      c.refine_stop = NS_STOP_REFINE_STALL;
      break;
    }
    wg_update<T, NW, GR>(n, G, ldg, false, alpha, r, theta);
    ++refine;
  }
  c.refine_steps = refine;
  return c.refine_stop == NS_STOP_RESID_TOL;
}


// A float64 leader's team context (ts == nullptr: products run on the
// workgroup alone).
struct TeamCtx {
  TeamState* ts;
  int* bc;          // LDS broadcast slot
  int32_t* err;     // the submission's error flag
  double* part;     // per-block partial sums (global, the leader's slot)
  int64_t ticks_ms; // device wall-clock ticks per millisecond
};

// Leader: one product shared with the team.  Publishes the phase, computes
// blocks until none is left to claim, waits for the blocks others claimed,
// then sums the per-block partial sums in block order (the result does not
// depend on who computed which block).
template <int NW>
__device__ double team_gemm(const TeamCtx& tc, int n, const double* X, int ldx,
                            const double* XA, int64_t lda, const double* Y, int ldy, double* D,
                            int ldd, const double* E1, const double* E2, int lde, double diag,
                            double scale, bool want_ss, double* red, void* lds) {
  TeamState* ts = tc.ts;
  const int total = wg_gemm_blocks<double, NW>(n);
  if (threadIdx.x == 0) {
    TeamDesc& q = ts->desc;
    const uint32_t seq = q.seq + 1;
    q.X = X;
    q.XA = XA;
    q.Y = Y;
    q.D = D;
    q.E1 = E1;
    q.E2 = E2;
    q.part = tc.part;
    q.lda = lda;
    q.diag = diag;
    q.scale = scale;
    q.n = n;
    q.ldx = ldx;
    q.ldy = ldy;
    q.ldd = ldd;
    q.lde = lde;
    q.total = total;
    q.want_ss = want_ss ? 1 : 0;
    q.seq = seq;
    __hip_atomic_store(&ts->done, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    fence_rel();   // the descriptor and operands before the phase opens
    __hip_atomic_store(&ts->claim, (unsigned long long)seq << 32, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (;;) {
    if (threadIdx.x == 0) tc.bc[0] = (int)(atomicAdd(&ts->claim, 1ULL) & 0xffffffffULL);
    __syncthreads();
    const int blk = tc.bc[0];
    __syncthreads();
    if (blk >= total) break;
    const double sl = wg_gemm_block<double, NW>(blk, n, X, ldx, XA, lda, Y, ldy, D, ldd, E1, E2,
                                                lde, diag, scale, lds);
    const double bs = want_ss ? block_sum_all<NW>(sl, red) : 0.0;
    if (threadIdx.x == 0) {
      if (want_ss) tc.part[blk] = bs;
      fence_rel();
      atomicAdd(&ts->done, 1);
    }
  }
  if (threadIdx.x == 0) {
    // Blocks claimed by others are being computed by running workgroups
    // that wait for nothing, so this wait ends; the bound only guards it.
    const int64_t t0 = wall_clock64();
    while (ld_rlx(&ts->done) < total) {
      __builtin_amdgcn_s_sleep(2);
      if (wall_clock64() - t0 > kWaitMs * tc.ticks_ms) {
        atomicExch(tc.err, 1);
        break;
      }
    }
    fence_acq();   // every block of the product, whoever wrote it
  }
  __syncthreads();
  double ss = 0.0;
  if (want_ss) {
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int b = 0; b < total; ++b)   // written by other workgroups: atomic loads
        t += __hip_atomic_load(tc.part + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      red[0] = t;
    }
    __syncthreads();
    ss = red[0];
    __syncthreads();
  }
  return ss;
}

// Field-by-field atomic copy of a team descriptor written by another
// workgroup (atomic loads are never served from the scalar cache).
__device__ __forceinline__ void load_desc(const TeamDesc* g, TeamDesc* l) {
  const uint64_t* src = reinterpret_cast<const uint64_t*>(g);
  uint64_t* dst = reinterpret_cast<uint64_t*>(l);
  static_assert(sizeof(TeamDesc) % 8 == 0, "descriptor copied in 8-byte words");
  for (int i = 0; i < (int)(sizeof(TeamDesc) / 8); ++i)
    dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Helper: compute blocks of team ts's current product while it has blocks
// left to claim.  Never waits: a failed claim ends the help.  sdesc: LDS
// copy of the descriptor.
template <int NW>
__device__ void team_help(TeamState* ts, double* red, void* lds, int* bc, TeamDesc* sdesc) {
  for (;;) {
    if (threadIdx.x == 0) {
      int got = -1;
      unsigned long long c = ld_rlx64(&ts->claim);
      for (int tries = 0; tries < 8; ++tries) {
        const uint32_t ph = (uint32_t)(c >> 32), j = (uint32_t)c;
        const uint32_t dseq = __hip_atomic_load(&ts->desc.seq, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
        const int total = __hip_atomic_load(&ts->desc.total, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        if (ph == 0 || dseq != ph || (int)j >= total) break;
        // Succeeds only while phase ph still has block j unclaimed, so the
        // descriptor read above is the phase's own (it changes only after
        // every block of the phase is done).
        const unsigned long long prev = atomicCAS(&ts->claim, c, c + 1);
        if (prev == c) {
          got = (int)j;
          break;
        }
        c = prev;
      }
      bc[0] = got;
    }
    if (threadIdx.x == 0 && bc[0] >= 0) {
      fence_acq();   // the phase's descriptor and operands, written before it opened
      load_desc(&ts->desc, sdesc);
    }
    __syncthreads();
    const int blk = bc[0];
    __syncthreads();
    if (blk < 0) return;
    const TeamDesc q = *sdesc;
    const double sl = wg_gemm_block<double, NW>(blk, q.n, q.X, q.ldx, q.XA, q.lda, q.Y, q.ldy,
                                                q.D, q.ldd, q.E1, q.E2, q.lde, q.diag, q.scale,
                                                lds);
    const double bs = q.want_ss ? block_sum_all<NW>(sl, red) : 0.0;
    if (threadIdx.x == 0) {
      if (q.want_ss) q.part[blk] = bs;
      fence_rel();
      atomicAdd(&ts->done, 1);
    }
  }
}

// A product of wg_solve: shared with the team (TEAM: a float64 leader of the
// escalating kernel), on the workgroup alone otherwise.
template <typename T, int NW, bool TEAM>
__device__ __forceinline__ double wg_mm(const TeamCtx& tc, int n, const T* X, int ldx,
                                        const double* XA, int64_t lda, const T* Y, int ldy, T* D,
                                        int ldd, const T* E1, const T* E2, int lde, T diag,
                                        T scale, bool want_ss, double* red, void* lds) {
  if constexpr (TEAM && sizeof(T) == 8) {
    return team_gemm<NW>(tc, n, X, ldx, XA, lda, Y, ldy, D, ldd, E1, E2, lde, diag, scale,
                         want_ss, red, lds);
  } else {
    return wg_gemm<T, NW>(n, X, ldx, XA, lda, Y, ldy, D, ldd, E1, E2, lde, diag, scale, want_ss,
                          red, lds);
  }
}

// One complete solve of system d in precision T.  Returns true when the
// refinement reached resid_tol.  hist: LDS history of ||F_k||_F (thread 0
// writes).  TEAM: a float64 leader whose products are shared through tc.
template <typename T, int NW, bool TEAM = false>
__device__ bool wg_solve(const BatchArgs& P, const BatchDesc& d, const SlotMats& sm, double* red,
                         double* hist, Ctl& c, const TeamCtx& tc = TeamCtx{}) {
  const int n = d.n, ldw = P.ldw;
  T* G[2] = {(T*)sm.G[0], (T*)sm.G[1]};
  T* F = (T*)sm.F;
  T* Pw[2] = {(T*)sm.P[0], (T*)sm.P[1]};
  T* Cc[2] = {(T*)sm.C[0], (T*)sm.C[1]};
  const bool is32 = sizeof(T) == 4;
  c.precision = is32 ? NS_PREC_FP32 : NS_PREC_FP64;
  c.mmm = 0;
  c.n_fnorm = 0;
  c.ns_steps = 0;
  c.refine_steps = 0;
  c.rel_resid = NAN;
  const double* sd = (P.scale == NS_SCALE_DIAG) ? sm.sd : nullptr;
  const double alpha = wg_alpha<NW>(P, d, red, sm.sd);
  c.alpha = alpha;
  if (!(alpha > 0.0) || !isfinite(alpha)) {
    c.ns_stop = NS_STOP_DIVERGED;
    c.refine_stop = NS_STOP_DIVERGED;
    return false;
  }
  if (is32) wg_copy_A<float, NW>(n, d.A, d.lda, sm.A32, ldw);  // for the residual products
  if (is32 && NSR_BATCH_F32_DMA) wg_zero_pads<NW>(n, sm.A32, ldw);  // K runs in whole slabs
  const T* AX = is32 ? (const T*)sm.A32 : nullptr;
  const double* AXd = is32 ? nullptr : d.A;
  // F_0 = I - A S^-1, theta_0 = S^-1 b, ||b||
  const double f0 = sqrt(wg_init_resid<T, NW>(n, d.A, d.lda, alpha, sd, F, ldw, red));
  const double bnorm = wg_theta0<NW>(n, d.b, d.theta, alpha, sd, red);
  if (threadIdx.x == 0) hist[0] = f0;
  c.n_fnorm = 1;
  int sexp = 0;
  while ((1 << sexp) < P.ns_order) ++sexp;
  bool implicit = true;
  int gc = 0;
  int ns_stop = isfinite(f0) ? NS_STOP_NONE : NS_STOP_DIVERGED;
  bool f2_ready = false;  // Pw[0] holds F_k^2 from the floor test
  // A float32 attempt that can escalate gives up at bail_step (see there).
  const int bail_k = (is32 && P.escalate) ? bail_step(P.ns_order) : 0;
  double fprev = f0;
  int k = 0;
  while (ns_stop == NS_STOP_NONE) {
    ++k;
    // C with P(F) = I + C (identity-offset squaring form).
    const T* pw = F;
    const T* cc = F;
    for (int i = 1; i < sexp; ++i) {
      T* npw = (pw == Pw[0]) ? Pw[1] : Pw[0];
      if (!(i == 1 && f2_ready)) {
        wg_mm<T, NW, TEAM>(tc, n, pw, ldw, nullptr, 0, pw, ldw, npw, ldw, nullptr, nullptr, ldw, T(0),
                       T(1), false, red, sm.lds);
        c.mmm += 1;
      }
      T* nc = (cc == Cc[0]) ? Cc[1] : Cc[0];
      wg_mm<T, NW, TEAM>(tc, n, cc, ldw, nullptr, 0, npw, ldw, nc, ldw, cc, npw, ldw, T(0), T(1), false,
                     red, sm.lds);
      c.mmm += 1;
      pw = npw;
      cc = nc;
    }
    T* Gn = G[gc ^ 1];
    if (implicit) {
      wg_scaled_identity_plus<T, NW>(n, cc, alpha, sd, Gn, ldw);
    } else {
      wg_mm<T, NW, TEAM>(tc, n, G[gc], ldw, nullptr, 0, cc, ldw, Gn, ldw, G[gc], nullptr, ldw, T(0), T(1),
                     false, red, sm.lds);
      c.mmm += 1;
    }
    gc ^= 1;
    implicit = false;
    // Richardson with G_k (eq. redttk1)
    wg_resid<NW, NSR_BATCH_GR>(n, d.A, d.lda, d.b, d.theta, sm.r, red);
    wg_update<T, NW, NSR_BATCH_GR>(n, G[gc], ldw, false, alpha, sm.r, d.theta);
    // F_k = I - A G_k
    const double fk =
        sqrt(wg_mm<T, NW, TEAM>(tc, n, AX, ldw, AXd, d.lda, G[gc], ldw, F, ldw, nullptr, nullptr, ldw,
                            T(1), T(-1), true, red, sm.lds));
    c.mmm += 1;
    if (threadIdx.x == 0 && k < NS_HIST_F) hist[k] = fk;
    c.n_fnorm = (k + 1 < NS_HIST_F) ? k + 1 : NS_HIST_F;
    // Stop rule: divergence, tolerance, rounding floor (||F_k|| > ||F_{k-1}||/2
    // although ||F_k^2|| <= ||F_k|| / 4, impossible in exact arithmetic), k_max.
    f2_ready = false;
    if (!isfinite(fk) || fk > f0) {
      ns_stop = NS_STOP_DIVERGED;
    } else if (fk <= P.f_tol) {
      ns_stop = NS_STOP_F_TOL;
    } else if (bail_k > 0 && k >= bail_k && fk >= 0.5 && fk > 0.5 * fprev) {
      // Every eigenvalue float32 can tell from 1 (mu <= 1 - 2^-24) is below
      // 2^-(order^2) by now; a norm still >= 1/2 that does not halve belongs
      // to eigenvalues float32 rounds to 1.
      ns_stop = NS_STOP_PRECISION;
    } else if (P.floor_detect && fprev < 1.0 && fk > kLawMargin * pow(fprev, (double)P.ns_order)) {
      // Error law (eq. fk1): ||F_k|| <= ||F_{k-1}||^n in exact arithmetic; a
      // norm far above it is rounding error: floor.
      ns_stop = NS_STOP_FLOOR;
    } else {
      if (P.floor_detect && fk > 0.5 * fprev) {
        const double f2 = sqrt(wg_mm<T, NW, TEAM>(tc, n, F, ldw, nullptr, 0, F, ldw, Pw[0], ldw, nullptr,
                                              nullptr, ldw, T(0), T(1), true, red, sm.lds));
        c.mmm += 1;
        f2_ready = true;
        if (f2 <= 0.25 * fk) ns_stop = NS_STOP_FLOOR;
      }
      if (ns_stop == NS_STOP_NONE && k >= P.k_max) ns_stop = NS_STOP_K_MAX;
    }
    fprev = fk;
  }
  c.ns_steps = k;
  c.ns_stop = ns_stop;
  if (ns_stop == NS_STOP_DIVERGED) {
    c.refine_stop = NS_STOP_DIVERGED;
    return false;
  }
  if (ns_stop == NS_STOP_PRECISION) {
    c.refine_stop = NS_STOP_NONE;
    return false;
  }
  return wg_refine<T, NW, NSR_BATCH_GR>(P, n, d.A, d.lda, d.b, d.theta, G[gc], ldw, alpha, sm.r,
                                        bnorm, red, c);
}

// ---------------------------------------------------------------------------
// Small systems (n <= SMALL_N, orders 2 and 4): the whole iteration in LDS.
// Four n x n matrices live in the workgroup's LDS (two G buffers, F, C); the
// GEMMs read their MFMA operands straight from LDS, so a step costs no global
// traffic beyond A, b and theta.  For order 4, F^2 is formed in the G buffer
// that G_{k+1} overwrites afterwards, and A (in precision T) is staged into
// C's buffer for the residual product once C is consumed.  Matrices are
// zero-padded to a multiple of 16 and every writer stores only the n x n
// part, so the 16 x 16 MFMA blocks need no edge handling.
// ---------------------------------------------------------------------------
constexpr int SMALL_N = 64;
template <typename T> struct SmallLd {
  static constexpr int value = SMALL_N + (sizeof(T) == 8 ? 2 : 4);   // row stride
};

// D = diag I + scale X Y + E1 + E2 over the padded size np, all in LDS at
// element offsets of `lds` (row stride SmallLd; e1 / e2 < 0: no addend);
// returns sum D^2 when want_ss (uniform).  Offsets rather than pointers keep
// every access a known LDS access (a pointer chosen at run time between two
// LDS buffers compiles to flat loads).  Every wave takes up to 16 / NW 16 x 16
// blocks (np = 64 fills them exactly; smaller np repeats blocks, whose results
// are dropped).
template <typename T, int NW>
__device__ double lds_gemm(T* lds, int np, int n, int xo, int yo, int dout, int e1, int e2,
                           T diag, T scale, bool want_ss, double* red) {
  typedef typename Acc<T>::type acc_t;
  constexpr int LD = SmallLd<T>::value;
  constexpr int MAXF = 16 / NW;
  static_assert(NW == 4 || NW == 8, "small-system GEMM runs on four or eight waves");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nf = np >> 4, nfrag = nf * nf;
  int x0[MAXF], y0[MAXF];
#pragma unroll
  for (int u = 0; u < MAXF; ++u) {
    const int f = (wave + u * NW) % nfrag;
    x0[u] = xo + ((f / nf) * 16 + lr) * LD + lk;   // X[row][k + lk]
    y0[u] = yo + lk * LD + (f % nf) * 16 + lr;     // Y[k + lk][col]
  }
  acc_t acc[MAXF];
#pragma unroll
  for (int u = 0; u < MAXF; ++u) acc[u] = acc_t{0, 0, 0, 0};
  // 16 values of k per round: all operand reads of the round are issued
  // before its MFMAs, so the round waits for LDS once.
  for (int k0 = 0; k0 < np; k0 += 16) {
    T a[4][MAXF], b[4][MAXF];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int u = 0; u < MAXF; ++u) {
        a[kk][u] = lds[x0[u] + k0 + 4 * kk];
        b[kk][u] = lds[y0[u] + (k0 + 4 * kk) * LD];
      }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int u = 0; u < MAXF; ++u) acc[u] = mfma(a[kk][u], b[kk][u], acc[u]);
  }
  double ss = 0.0;
#pragma unroll
  for (int u = 0; u < MAXF; ++u) {
    const int f = wave + u * NW;
    if (f >= nfrag) continue;
    const int col = (f % nf) * 16 + lr;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = (f / nf) * 16 + acc_row(T(0), lk, r);
      if (row < n && col < n) {
        const int at = row * LD + col;
        T v = scale * acc[u][r];
        if (row == col) v += diag;
        if (e1 >= 0) v += lds[e1 + at];
        if (e2 >= 0) v += lds[e2 + at];
        lds[dout + at] = v;
        if (want_ss) ss += (double)v * (double)v;
      }
    }
  }
  __syncthreads();
  return want_ss ? block_sum_all<NW>(ss, red) : 0.0;
}

// Matrix-vector products of the LDS path (n <= SMALL_N; A, x, y in LDS):
// lane l of every wave takes row l over the wave's share of the columns, the
// NW partial sums of a row are added in wave order (part: NW x SMALL_N
// float64 of LDS).  No cross-lane reduction: a shuffle tree per row would be
// a chain of dependent LDS permutes.
// r = b - A theta; returns ||r||^2 (uniform).
template <int NW>
__device__ double small_resid(int n, const double* A, int lda, const double* b,
                              const double* theta, double* r, double* part, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cw = (n + NW - 1) / NW, c0 = wave * cw, c1 = min(n, c0 + cw);
  if (lane < n) {
    double s = 0.0;
    for (int c = c0; c < c1; ++c) s += A[lane * lda + c] * theta[c];
    part[wave * SMALL_N + lane] = s;
  }
  __syncthreads();
  double ss = 0.0;
  if (wave == 0 && lane < n) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += part[w * SMALL_N + lane];
    const double rv = b[lane] - s;
    r[lane] = rv;
    ss = rv * rv;
  }
  return block_sum_all<NW>(ss, red);
}

// theta += G r.
template <typename T, int NW>
__device__ void small_update(int n, const T* G, int ldg, const double* r, double* theta,
                             double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int cw = (n + NW - 1) / NW, c0 = wave * cw, c1 = min(n, c0 + cw);
  if (lane < n) {
    double s = 0.0;
    for (int c = c0; c < c1; ++c) s += (double)G[lane * ldg + c] * r[c];
    part[wave * SMALL_N + lane] = s;
  }
  __syncthreads();
  if (wave == 0 && lane < n) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += part[w * SMALL_N + lane];
    theta[lane] += s;
  }
  __syncthreads();
}

// Richardson refinement of the LDS path (as wg_refine).
template <typename T, int NW>
__device__ bool small_refine(const BatchArgs& P, int n, const double* A, int lda,
                             const double* b, double* theta, const T* G, int ldg, double* r,
                             double* part, double bnorm, double* red, Ctl& c) {
  double last[4] = {0, 0, 0, 0};
  int refine = 0;
  while (true) {
    const double rel = sqrt(small_resid<NW>(n, A, lda, b, theta, r, part, red)) / bnorm;
    c.rel_resid = rel;
    for (int j = 3; j > 0; --j) last[j] = last[j - 1];
    last[0] = rel;
    if (!isfinite(rel)) {
      c.refine_stop = NS_STOP_DIVERGED;
      break;
    }
    if (rel <= P.resid_tol) {
      c.refine_stop = NS_STOP_RESID_TOL;
      break;
    }
    if (refine >= P.refine_max) {
      c.refine_stop = NS_STOP_REFINE_MAX;
      break;
    }
    if (refine >= 3 && rel > 0.5 * last[3]) {
      c.refine_stop = NS_STOP_REFINE_STALL;
      break;
    }
    small_update<T, NW>(n, G, ldg, r, theta, part);
    ++refine;
  }
  c.refine_steps = refine;
  return c.refine_stop == NS_STOP_RESID_TOL;
}

// One complete solve of a small system in LDS (same steps, stop rule and
// escalation as wg_solve; orders 2 and 4).  lds: the four matrices (two G
// buffers, F, C; SMALL_N x SmallLd elements each).  vec: 4 x SMALL_N float64
// of LDS for theta, b and the residual; theta goes to global memory at the
// end.  A in float64: a64 (float32 solves; copied once, leading dimension
// SMALL_N) or, in float64 solves, C's buffer, refilled every step once C is
// consumed; the residual products read A in precision T from C's buffer.
// part: NW x SMALL_N float64 of LDS for the matrix-vector products.
template <typename T, int NW>
__device__ bool wg_solve_small(const BatchArgs& P, const BatchDesc& d, T* lds, double* vec,
                               double* a64, double* part, double* red, double* hist, Ctl& c) {
  constexpr int LD = SmallLd<T>::value;
  constexpr int MS = SMALL_N * LD;   // elements per matrix
  constexpr bool dbl = sizeof(T) == 8;
  const int n = d.n, np = (n + 15) & ~15;
  const int oG[2] = {0, MS};
  const int oF = 2 * MS, oC = 3 * MS;
  double* th = vec;
  double* bv = vec + SMALL_N;
  double* rv = vec + 2 * SMALL_N;
  double* sv = vec + 3 * SMALL_N;   // S = diag(A) (NS_SCALE_DIAG)
  const double* sd = (P.scale == NS_SCALE_DIAG) ? sv : nullptr;
  // float64 A: C's buffer (float64 solves) or a64
  double* A64 = dbl ? reinterpret_cast<double*>(lds) + oC : a64;
  constexpr int ALD = dbl ? LD : SMALL_N;
  c.precision = dbl ? NS_PREC_FP64 : NS_PREC_FP32;
  c.mmm = 0;
  c.n_fnorm = 0;
  c.ns_steps = 0;
  c.refine_steps = 0;
  c.rel_resid = NAN;
  for (int i = threadIdx.x; i < 4 * MS; i += NW * 64) lds[i] = T(0);
  for (int i = threadIdx.x; i < n; i += NW * 64) bv[i] = d.b[i];
  __syncthreads();
  const double alpha = wg_alpha<NW>(P, d, red, sv);
  c.alpha = alpha;
  if (!(alpha > 0.0) || !isfinite(alpha)) {
    c.ns_stop = NS_STOP_DIVERGED;
    c.refine_stop = NS_STOP_DIVERGED;
    return false;
  }
  wg_copy_A<double, NW>(n, d.A, d.lda, A64, ALD);
  const double f0 = sqrt(wg_init_resid<T, NW>(n, A64, ALD, alpha, sd, lds + oF, LD, red));
  const double bnorm = wg_theta0<NW>(n, bv, th, alpha, sd, red);
  if (threadIdx.x == 0) hist[0] = f0;
  c.n_fnorm = 1;
  const bool order4 = P.ns_order == 4;
  const int bail_k = (!dbl && P.escalate) ? bail_step(P.ns_order) : 0;
  bool implicit = true, f2_ready = false;
  int gc = 0, k = 0;
  int ns_stop = isfinite(f0) ? NS_STOP_NONE : NS_STOP_DIVERGED;
  double fprev = f0;
  while (ns_stop == NS_STOP_NONE) {
    ++k;
    // C with P(F) = I + C: order 4, C = F + F^2 + F F^2 (F^2 in the G buffer
    // that receives G_{k+1}); order 2, C = F.
    const int oGn = oG[gc ^ 1];
    int occ = oF;
    if (order4) {
      if (!f2_ready) {
        lds_gemm<T, NW>(lds, np, n, oF, oF, oGn, -1, -1, T(0), T(1), false, red);
        c.mmm += 1;
      }
      lds_gemm<T, NW>(lds, np, n, oF, oGn, oC, oF, oGn, T(0), T(1), false, red);
      c.mmm += 1;
      occ = oC;
    }
    if (implicit) {
      wg_scaled_identity_plus<T, NW>(n, lds + occ, alpha, sd, lds + oGn, LD);
    } else {
      lds_gemm<T, NW>(lds, np, n, oG[gc], occ, oGn, oG[gc], -1, T(0), T(1), false, red);
      c.mmm += 1;
    }
    gc ^= 1;
    implicit = false;
    // A into C's buffer: float64 (float64 solves) or, from a64, float32
    if (dbl)
      wg_copy_A<double, NW>(n, d.A, d.lda, A64, ALD);
    else
      wg_copy_A<T, NW>(n, A64, ALD, lds + oC, LD);
    // Richardson with G_k (eq. redttk1)
    small_resid<NW>(n, A64, ALD, bv, th, rv, part, red);
    small_update<T, NW>(n, lds + oG[gc], LD, rv, th, part);
    // F_k = I - A G_k
    const double fk =
        sqrt(lds_gemm<T, NW>(lds, np, n, oC, oG[gc], oF, -1, -1, T(1), T(-1), true, red));
    c.mmm += 1;
    if (threadIdx.x == 0 && k < NS_HIST_F) hist[k] = fk;
    c.n_fnorm = (k + 1 < NS_HIST_F) ? k + 1 : NS_HIST_F;
    f2_ready = false;
    if (!isfinite(fk) || fk > f0) {
      ns_stop = NS_STOP_DIVERGED;
    } else if (fk <= P.f_tol) {
      ns_stop = NS_STOP_F_TOL;
    } else if (bail_k > 0 && k >= bail_k && fk >= 0.5 && fk > 0.5 * fprev) {
      ns_stop = NS_STOP_PRECISION;
    } else if (P.floor_detect && fprev < 1.0 && fk > kLawMargin * pow(fprev, (double)P.ns_order)) {
      ns_stop = NS_STOP_FLOOR;   // error law, as in wg_solve
    } else {
      if (P.floor_detect && fk > 0.5 * fprev) {
        // F_k^2 goes to the G buffer G_{k+1} will overwrite (it holds G_{k-1}).
        const double f2 = sqrt(lds_gemm<T, NW>(lds, np, n, oF, oF, oG[gc ^ 1], -1, -1, T(0),
                                               T(1), true, red));
        c.mmm += 1;
        f2_ready = order4;
        if (f2 <= 0.25 * fk) ns_stop = NS_STOP_FLOOR;
      }
      if (ns_stop == NS_STOP_NONE && k >= P.k_max) ns_stop = NS_STOP_K_MAX;
    }
    fprev = fk;
  }
  c.ns_steps = k;
  c.ns_stop = ns_stop;
  bool ok = false;
  if (ns_stop == NS_STOP_DIVERGED) {
    c.refine_stop = NS_STOP_DIVERGED;
  } else if (ns_stop == NS_STOP_PRECISION) {
    c.refine_stop = NS_STOP_NONE;
  } else {
    ok = small_refine<T, NW>(P, n, A64, ALD, bv, th, lds + oG[gc], LD, rv, part, bnorm, red, c);
  }
  for (int i = threadIdx.x; i < n; i += NW * 64) d.theta[i] = th[i];
  __syncthreads();
  return ok;
}

// Report of one attempt (thread 0).  The float32 pass queues a system it
// could not solve for the float64 pass when escalation is on.
__device__ __forceinline__ void write_result(const BatchArgs& P, int sid, bool dbl, bool from_queue, bool ok,
                             Ctl c, const double* hist, int64_t t_begin) {
  BatchResult* R = &P.res[sid];
  const int slot_t = dbl ? 2 : 0;
  R->clock[slot_t] = t_begin;
  R->clock[slot_t + 1] = wall_clock64();
  R->wg[dbl ? 1 : 0] = blockIdx.x;
  if (!from_queue) {   // first attempt of this system: clear the other one
    R->clock[2 - slot_t] = 0;
    R->clock[3 - slot_t] = 0;
    R->wg[dbl ? 0 : 1] = -1;
  }
  if (from_queue) c.mmm += R->mmm;   // the float32 attempt's products
  R->status = ok ? NS_OK
                 : ((c.ns_stop == NS_STOP_DIVERGED || c.refine_stop == NS_STOP_DIVERGED)
                        ? NS_EDIVERGED
                        : NS_ENOCONV);
  R->ns_stop = c.ns_stop;
  R->refine_stop = c.refine_stop;
  R->ns_steps = c.ns_steps;
  R->refine_steps = c.refine_steps;
  R->precision = c.precision;
  R->n_fnorm = c.n_fnorm;
  R->n_resid = 0;
  R->alpha = c.alpha;
  R->rel_resid = c.rel_resid;
  R->mmm = c.mmm;
  for (int j = 0; j < c.n_fnorm; ++j) R->fnorm_hist[j] = hist[j];
  if (!dbl && !ok && P.escalate) {
    // Queue the system for float64: the result record above is written
    // first (release fence), then the entry (sid + 1) is published.
    fence_rel();
    const int idx = atomicAdd(P.counter + 2, 1);
    __hip_atomic_store(P.retry + idx, sid + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // Float32 attempts finished.  Not ordered after a push: a team workgroup
  // that sees the count before the entry only exits early, and the float64
  // pass that follows on the float32 pass's stream re-solves what is left.
  if (!dbl) atomicAdd(P.counter + 4, 1);
}

// Persistent solver: each workgroup pulls systems from a work counter (the
// host sorted them largest first) and solves each one completely.  The
// float32 pass (T = float) queues the systems it cannot bring to the
// tolerance in P.retry when escalation is on; the float64 pass (T = double)
// then re-solves the queued systems (or, in float64-only mode, all systems).
// The two precisions are separate kernels so that each gets the register
// budget of its own solve.
// Slot of one workgroup: 8 float32 matrices (A in float32, G x 2, F, P x 2,
// C x 2), 7 float64 matrices (G x 2, F, P x 2, C x 2), the residual vector
// and the per-block partial sums of a float64 team product, each n x n
// matrix with leading dimension ldw.
template <typename T>
__device__ __forceinline__ SlotMats slot_mats(const BatchArgs& P, char* slot, void* lds) {
  const int64_t nn = (int64_t)P.ldw * P.ldw;
  float* f = reinterpret_cast<float*>(slot);
  double* d = reinterpret_cast<double*>(f + 8 * nn);
  SlotMats sm;
  if (sizeof(T) == 4) {
    sm.A32 = f;
    sm.G[0] = f + nn;
    sm.G[1] = f + 2 * nn;
    sm.F = f + 3 * nn;
    sm.P[0] = f + 4 * nn;
    sm.P[1] = f + 5 * nn;
    sm.C[0] = f + 6 * nn;
    sm.C[1] = f + 7 * nn;
  } else {
    sm.A32 = nullptr;
    sm.G[0] = d;
    sm.G[1] = d + nn;
    sm.F = d + 2 * nn;
    sm.P[0] = d + 3 * nn;
    sm.P[1] = d + 4 * nn;
    sm.C[0] = d + 5 * nn;
    sm.C[1] = d + 6 * nn;
  }
  sm.r = d + 7 * nn;
  sm.sd = d + 7 * nn + P.ldw;
  sm.lds = lds;
  return sm;
}

__device__ __forceinline__ double* slot_part(const BatchArgs& P, char* slot) {
  const int64_t nn = (int64_t)P.ldw * P.ldw;
  return reinterpret_cast<double*>(slot + 8 * nn * sizeof(float)) + 7 * nn + 2 * P.ldw;
}

template <typename T, int NW>
__device__ __forceinline__ void batch_loop(const BatchArgs& P, double* red, double* hist,
                                           int& s_idx, char* stage) {
  constexpr bool dbl = sizeof(T) == 8;
  char* slot = P.slots + (int64_t)(P.slot_base + blockIdx.x) * P.slot_bytes;
  const SlotMats sm = slot_mats<T>(P, slot, stage);
  // Work list: all systems in P.order, or (float64 after float32) the queue
  // (after a lockstep re-solve: its overflow queue).
  const bool from_queue = dbl && !P.fp64_only;
  const bool ovf = from_queue && P.ls_on;
  int* counter = P.counter + (ovf ? 6 : (from_queue ? 1 : 0));
  const int total = ovf ? P.counter[7] : (from_queue ? P.counter[2] : P.count);
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int q = s_idx;
    __syncthreads();
    if (q >= total) break;
    const int sid = ovf ? P.ovf[q] - 1 : (from_queue ? P.retry[q] - 1 : P.order[q]);
    const BatchDesc d = P.desc[sid];
    const int64_t t_begin = wall_clock64();
    Ctl c;
    const bool ok = wg_solve<T, NW>(P, d, sm, red, hist, c);
    __syncthreads();  // hist complete
    if (threadIdx.x == 0) write_result(P, sid, dbl, from_queue, ok, c, hist, t_begin);
    __syncthreads();
  }
}


// Held to 128 registers per lane (four waves per SIMD, two eight-wave
// workgroups per CU): the solve then spills some 40 registers (loop-invariant
// addresses) to scratch, and still runs the 2048-system batch 13% (float32
// pass) to 15% (float64-only) faster than at two waves per SIMD unspilled.
template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4)))
batch_kernel(BatchArgs P) {
  __shared__ double red[NW];
  __shared__ double hist[NS_HIST_F];
  __shared__ int s_idx;
  __shared__ __attribute__((aligned(1024))) char stage[StageBytes<T, NW>::value];
  batch_loop<T, NW>(P, red, hist, s_idx, stage);
}

// The float32 pass of an escalating submission: batch_kernel<float, NW> held
// to at most a third of a SIMD's registers per wave, so that a workgroup of
// team_kernel (same bound, one wave per SIMD) is resident beside an
// eight-wave workgroup of this pass on every compute unit.
template <int NW>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(3)))
f32_pass_kernel(BatchArgs P) {
  __shared__ double red[NW];
  __shared__ double hist[NS_HIST_F];
  __shared__ int s_idx;
  __shared__ __attribute__((aligned(1024))) char stage[StageBytes<float, NW>::value];
  batch_loop<float, NW>(P, red, hist, s_idx, stage);
}

// Float64 re-solves of the systems the float32 pass queues, running beside
// that pass (on another stream, launched with it).  Its workgroups are small
// enough to be resident on the same compute units as the float32 pass's.
// Each repeats, in this order of priority:
//  1. claim a queued system and re-solve it in float64 as the leader of its
//     team (its products shared, block by block, with idle workgroups);
//  2. help a team: compute blocks of its current product;
//  3. otherwise sleep briefly; exit once the float32 pass has finished every
//     attempt (so nothing more is queued) and every claimed re-solve is done.
// Only two waits exist, both on work held by running workgroups that wait
// for nothing: a leader for the blocks others claimed, and a claimer for the
// queue entry whose producer is between its two writes; both are bounded.
// Helping is optional and a workgroup with nothing to do may always exit
// (after kIdleLimit rounds): entries it leaves unclaimed are re-solved by the
// float64 pass that follows on the float32 pass's stream.
template <int NW>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(3)))
team_kernel(BatchArgs P) {
  __shared__ double red[NW];
  __shared__ double hist[NS_HIST_F];
  __shared__ int bc[4];
  __shared__ TeamDesc sdesc;
  __shared__ __attribute__((aligned(16))) char stage[Stage<double, NW>::BYTES];
  char* slot = P.slots + (int64_t)(P.slot_base + blockIdx.x) * P.slot_bytes;
  const SlotMats s64 = slot_mats<double>(P, slot, stage);
  double* part = slot_part(P, slot);
  int32_t* cnt = P.counter;
  const int64_t t_start = wall_clock64();
  int64_t t_work = t_start;   // last time this workgroup had work
  for (;;) {
    // 1. lead a queued float64 re-solve
    if (threadIdx.x == 0) {
      int arg = -1;
      const int qlen = ld_rlx(cnt + 2);
      int qc = ld_rlx(cnt + 1);
      while (qc < qlen) {
        const int prev = atomicCAS(cnt + 1, qc, qc + 1);
        if (prev == qc) {
          arg = qc;
          break;
        }
        qc = prev;
      }
      bc[0] = arg;
      bc[1] = qlen;
    }
    __syncthreads();
    const int q = bc[0], qlen = bc[1];
    __syncthreads();
    if (q >= 0) {
      if (threadIdx.x == 0) {
        // the producer is between its count and its entry write
        int v;
        while ((v = ld_rlx(P.retry + q)) == 0) {
          __builtin_amdgcn_s_sleep(1);
          if (wall_clock64() - t_work > kWaitMs * P.ticks_ms) {
            atomicExch(cnt + 5, 2);
            break;
          }
        }
        fence_acq();   // the float32 attempt's result record
        bc[2] = v - 1;
      }
      __syncthreads();
      const int sid = bc[2];
      __syncthreads();
      if (sid >= 0) {
        TeamState* ts = P.team + q;
        if (threadIdx.x == 0)
          __hip_atomic_store(&ts->active, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const BatchDesc d = P.desc[sid];
        const int64_t t_begin = wall_clock64();
        Ctl c;
        const bool ok =
            wg_solve<double, NW, true>(P, d, s64, red, hist, c,
                                       TeamCtx{ts, bc + 3, cnt + 5, part, P.ticks_ms});
        __syncthreads();
        if (threadIdx.x == 0) {
          __hip_atomic_store(&ts->active, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          write_result(P, sid, true, true, ok, c, hist, t_begin);
          atomicAdd(cnt + 3, 1);
        }
        __syncthreads();
      } else if (threadIdx.x == 0) {
        atomicAdd(cnt + 3, 1);
      }
      t_work = wall_clock64();
      continue;
    }
    // 2. help a team that has blocks left to claim (wave 0 scans the queue)
    if (qlen > 0 && threadIdx.x < 64) {
      int found = -1;
      for (int base = 0; base < qlen && found < 0; base += 64) {
        const int e = base + (int)threadIdx.x;
        bool has = false;
        if (e < qlen) {
          TeamState* ts = P.team + e;
          if (__hip_atomic_load(&ts->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            const unsigned long long c = ld_rlx64(&ts->claim);
            const int total =
                __hip_atomic_load(&ts->desc.total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            has = (c >> 32) != 0 && (int)(uint32_t)c < total;
          }
        }
        const unsigned long long m = __ballot(has);
        if (m) found = base + __builtin_ffsll((long long)m) - 1;
      }
      if (threadIdx.x == 0) bc[0] = found;
    }
    __syncthreads();
    const int h = bc[0];
    __syncthreads();
    if (h >= 0) {
      team_help<NW>(P.team + h, red, stage, bc + 3, &sdesc);
      t_work = wall_clock64();
      continue;
    }
    // 3. nothing to do now: exit once the float32 pass is over and every
    //    queued system is claimed and done, when idle for kIdleMs, or when
    //    the float32 pass has not started kStartMs after this kernel (the
    //    two kernels then run one after the other, and the float64 pass on
    //    the float32 pass's stream re-solves the queue); else wait a little
    if (threadIdx.x == 0) {
      const int64_t now = wall_clock64();
      const bool all = ld_rlx(cnt + 4) >= P.count && ld_rlx(cnt + 3) >= ld_rlx(cnt + 2);
      const bool stale = now - t_work > kIdleMs * P.ticks_ms ||
                         (ld_rlx(cnt) == 0 && now - t_start > kStartMs * P.ticks_ms);
      bc[0] = (all || stale) ? 1 : 0;
    }
    __syncthreads();
    const int stop = bc[0];
    __syncthreads();
    if (stop) break;
    __builtin_amdgcn_s_sleep(16);
  }
}

// Persistent solver for submissions whose systems all fit the LDS path
// (n <= SMALL_N, order 2 or 4); same work list, queue and reports as
// batch_kernel.

// ---------------------------------------------------------------------------
// Lockstep float64 re-solve of the queued systems.  The systems float32
// could not solve (the queue, whose length only the device knows) are
// re-solved together, one sub-step of the Newton-Schulz step at a time:
// each product is one launch whose workgroups share the output blocks of
// every queued system (wg_gemm_block), and small per-system kernels run the
// Richardson update, the stop rule and the refinement.  A hard system's
// float64 chain then runs on many CUs at once instead of one, and no
// workgroup ever waits for another: kernel boundaries order the sub-steps.
// The arithmetic is the one-workgroup solve's (same blocks, same K order);
// the sums of squares add per-block partial sums in block order.  Queue
// entry q uses slot q; entries beyond the slots, and systems still iterating
// after the enqueued steps, go to the overflow queue, which the
// one-workgroup float64 pass re-solves afterwards.
// ---------------------------------------------------------------------------
constexpr int kLsNW = 8;      // waves of the lockstep per-system kernels
#ifndef NSR_LS_GEMM_NW
#define NSR_LS_GEMM_NW 8
#endif
constexpr int kLsGemmNW = NSR_LS_GEMM_NW;   // waves of the lockstep product kernel
constexpr int kLsMinN = 128;    // smallest largest-system size that uses lockstep
constexpr int kLsMinCount = 512;  // smallest batch that uses lockstep: the fixed
                                  // schedule (170 launches) costs ~2 ms of host
                                  // enqueue and ~0.5 ms of device time, which a
                                  // serving-sized batch (<= 256 systems) pays
                                  // in latency even when nothing escalates
constexpr int kLsSteps = 28;  // Newton-Schulz steps enqueued (capped by k_max)
enum : int { kLsPow = 0, kLsAsm = 1, kLsGside = 2, kLsResid = 3, kLsProbe = 4 };

__device__ __forceinline__ int ls_count(const BatchArgs& P) {
  const int q = P.counter[2];
  return q < P.ls_slots ? q : P.ls_slots;
}
__device__ __forceinline__ char* ls_slot(const BatchArgs& P, int q) {
  return P.slots + (int64_t)q * P.slot_bytes;
}

// Operands of system s's product in phase ph (sub-step i of the power loop),
// following wg_solve's buffer rotation: the power loop starts from F each
// step, so power i goes to Pw[(i - 1) & 1] and assembly i to Cc[(i - 1) & 1].
struct LsOp {
  const double* X;
  const double* XA;
  const double* Y;
  double* D;
  const double* E1;
  const double* E2;
  int64_t lda;
  double diag, scale;
  bool ss, elem;
};

__device__ __forceinline__ bool ls_operands(const BatchArgs& P, const LsState& s,
                                            const SlotMats& sm, int ph, int i, LsOp& o) {
  if (!s.active) return false;
  int sexp = 0;
  while ((1 << sexp) < P.ns_order) ++sexp;
  // Buffer choices by selects (an indexed local array would live in
  // private memory).
  double* const F = (double*)sm.F;
  auto pw = [&](int j) { return (j & 1) ? (double*)sm.P[1] : (double*)sm.P[0]; };
  auto cc = [&](int j) { return (j & 1) ? (double*)sm.C[1] : (double*)sm.C[0]; };
  double* const Gcur = s.gc ? (double*)sm.G[1] : (double*)sm.G[0];
  double* const Gnew = s.gc ? (double*)sm.G[0] : (double*)sm.G[1];
  o = LsOp{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, 0.0, 1.0, false, false};
  if (ph == kLsPow) {
    if (i == 1 && s.f2_ready) return false;   // F^2 from the floor probe
    o.X = o.Y = (i == 1) ? F : pw(i - 2);
    o.D = pw(i - 1);
    return true;
  }
  if (ph == kLsAsm) {
    o.X = o.E1 = (i == 1) ? F : cc(i - 2);
    o.Y = o.E2 = pw(i - 1);
    o.D = cc(i - 1);
    return true;
  }
  if (ph == kLsGside) {
    o.Y = sexp > 1 ? cc(sexp - 2) : F;
    o.D = Gnew;
    if (s.implicit)
      o.elem = true;            // G_1 = S^-1 (I + C)
    else
      o.X = o.E1 = Gcur;        // G_{k+1} = G_k + G_k C
    return true;
  }
  if (ph == kLsResid) {
    const BatchDesc d = P.desc[s.sid];
    o.XA = d.A;
    o.lda = d.lda;
    o.Y = Gnew;
    o.D = F;
    o.diag = 1.0;
    o.scale = -1.0;
    o.ss = true;
    return true;
  }
  if (ph == kLsProbe && s.probe) {
    o.X = o.Y = F;
    o.D = pw(0);
    o.ss = true;
    return true;
  }
  return false;
}

// Per-block partial sums of D^2 of the residual product (part[0..)) and of
// the floor probe (part[ls_probe_off..)): blocks of the largest system each.
__device__ __forceinline__ int ls_probe_off(int ldw) {
  return ((ldw + Block<kLsGemmNW>::BM - 1) / Block<kLsGemmNW>::BM) *
         ((ldw + Block<kLsGemmNW>::BN - 1) / Block<kLsGemmNW>::BN);
}

// Sum of one product's per-block partial sums, in block order.
__device__ __forceinline__ double ls_sum_parts(const BatchArgs& P, int q, int n, int off) {
  constexpr int BM = Block<kLsGemmNW>::BM, BN = Block<kLsGemmNW>::BN;
  const double* part = slot_part(P, ls_slot(P, q)) + off;
  const int nb = ((n + BM - 1) / BM) * ((n + BN - 1) / BN);
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[b];
  return t;
}

// The stop rule of wg_solve after the residual product of step k (state s
// before this step's update): returns the stop (NS_STOP_NONE: none) and
// whether the floor probe F_k^2 is needed.  A pure function of s and the
// partial sums, so the probe launch and the control launch agree.
__device__ __forceinline__ int ls_rule(const BatchArgs& P, const LsState& s, double fk,
                                       bool& probe) {
  probe = false;
  if (!isfinite(fk) || fk > s.f0) return NS_STOP_DIVERGED;
  if (fk <= P.f_tol) return NS_STOP_F_TOL;
  if (P.floor_detect && s.fprev < 1.0 && fk > kLawMargin * pow(s.fprev, (double)P.ns_order))
    return NS_STOP_FLOOR;
  probe = P.floor_detect && fk > 0.5 * s.fprev;
  return NS_STOP_NONE;
}

// One lockstep product for every participating system: items (system,
// block) strided over the grid.  The residual launch also carries one
// Richardson-update item per system (it reads the same new G and writes
// theta, which no product reads).
__global__ void __launch_bounds__(kLsGemmNW * 64) ls_gemm_kernel(BatchArgs P, int ph, int i) {
  constexpr int NW = kLsGemmNW, BM = Block<NW>::BM, BN = Block<NW>::BN;
  __shared__ __attribute__((aligned(16))) char lds[Stage<double, NW>::BYTES];
  __shared__ double red[NW];
  const int nsys = ls_count(P);
  const int bmax = (P.ldw + BM - 1) / BM, bnmax = (P.ldw + BN - 1) / BN, per = bmax * bnmax;
  const int items = nsys * per + (ph == kLsResid ? nsys : 0);
  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    if (item >= nsys * per) {
      // Richardson update with G_k (eq. redttk1)
      const int q = item - nsys * per;
      const LsState s = P.ls[q];
      if (!s.active) continue;
      const BatchDesc d = P.desc[s.sid];
      const SlotMats sm = slot_mats<double>(P, ls_slot(P, q), nullptr);
      wg_resid<NW, NSR_BATCH_GR>(s.n, d.A, d.lda, d.b, d.theta, sm.r, red);
      wg_update<double, NW, NSR_BATCH_GR>(s.n, (const double*)(s.gc ? sm.G[0] : sm.G[1]), P.ldw,
                                          false, s.alpha, sm.r, d.theta);
      continue;
    }
    const int q = item / per, b = item % per;
    LsState s = P.ls[q];
    if (ph == kLsProbe && s.active) {
      bool probe;
      const double fk = sqrt(ls_sum_parts(P, q, s.n, 0));
      const int stop = ls_rule(P, s, fk, probe);
      s.probe = (stop == NS_STOP_NONE && probe) ? 1 : 0;
    }
    char* slot = ls_slot(P, q);
    const SlotMats sm = slot_mats<double>(P, slot, lds);
    LsOp o;
    if (!ls_operands(P, s, sm, ph, i, o)) continue;
    const int n = s.n, bi = b / bnmax, bj = b % bnmax;
    if (bi * BM >= n || bj * BN >= n) continue;
    const int blk = bi * ((n + BN - 1) / BN) + bj;
    if (o.elem) {
      // G_1 = S^-1 (I + C) over the block
      const double* sd = (P.scale == NS_SCALE_DIAG) ? sm.sd : nullptr;
      for (int e = threadIdx.x; e < BM * BN; e += NW * 64) {
        const int row = bi * BM + e / BN, col = bj * BN + e % BN;
        if (row < n && col < n) {
          double v = o.Y[row * P.ldw + col];
          if (row == col) v += 1.0;
          o.D[row * P.ldw + col] = v / (sd ? sd[row] : s.alpha);
        }
      }
      continue;
    }
    double ss = wg_gemm_block<double, NW>(blk, n, o.X, P.ldw, o.XA, o.lda, o.Y, P.ldw, o.D, P.ldw,
                                          o.E1, o.E2, P.ldw, o.diag, o.scale, lds);
    if (o.ss) {
      ss = block_sum_all<NW>(ss, red);
      if (threadIdx.x == 0)
        slot_part(P, slot)[(ph == kLsProbe ? ls_probe_off(P.ldw) : 0) + blk] = ss;
    }
  }
}

// Start of each queued system's float64 solve (F_0, theta_0), or its move
// to the overflow queue when the slots are taken.
__global__ void __launch_bounds__(kLsNW * 64) ls_init_kernel(BatchArgs P) {
  constexpr int NW = kLsNW;
  __shared__ double red[NW];
  const int qlen = P.counter[2];
  for (int q = blockIdx.x; q < qlen; q += gridDim.x) {
    const int sid = P.retry[q] - 1;
    if (q >= P.ls_slots) {
      if (threadIdx.x == 0) {
        const int idx = atomicAdd(P.counter + 7, 1);
        P.ovf[idx] = sid + 1;
      }
      continue;
    }
    const BatchDesc d = P.desc[sid];
    const SlotMats sm = slot_mats<double>(P, ls_slot(P, q), nullptr);
    const int64_t t0 = wall_clock64();
    const double* sd = (P.scale == NS_SCALE_DIAG) ? sm.sd : nullptr;
    const double alpha = wg_alpha<NW>(P, d, red, sm.sd);
    LsState st{};
    st.alpha = alpha;
    st.sid = sid;
    st.n = d.n;
    st.t_begin = t0;
    st.implicit = 1;
    st.ns_stop = NS_STOP_DIVERGED;
    if (alpha > 0.0 && isfinite(alpha)) {
      const double f0 =
          sqrt(wg_init_resid<double, NW>(d.n, d.A, d.lda, alpha, sd, (double*)sm.F, P.ldw, red));
      st.bnorm = wg_theta0<NW>(d.n, d.b, d.theta, alpha, sd, red);
      st.f0 = st.fprev = f0;
      st.ns_stop = isfinite(f0) ? NS_STOP_NONE : NS_STOP_DIVERGED;
      if (threadIdx.x == 0) P.res[sid].fnorm_hist[0] = f0;
    }
    st.active = st.ns_stop == NS_STOP_NONE;
    if (threadIdx.x == 0) P.ls[q] = st;
    __syncthreads();
  }
}

// End of a step (one thread per system): ||F_k||, its history, the stop
// rule with the floor probe's verdict, k_max, and the state for the next
// step.
__global__ void __launch_bounds__(64) ls_ctl_kernel(BatchArgs P) {
  const int nsys = ls_count(P);
  for (int q = blockIdx.x * 64 + threadIdx.x; q < nsys; q += gridDim.x * 64) {
    LsState s = P.ls[q];
    if (!s.active) continue;
    int sexp = 0;
    while ((1 << sexp) < P.ns_order) ++sexp;
    const double fk = sqrt(ls_sum_parts(P, q, s.n, 0));
    bool probe;
    int stop = ls_rule(P, s, fk, probe);
    s.k += 1;
    s.mmm += (sexp > 1 ? 2 * (sexp - 1) - (s.f2_ready ? 1 : 0) : 0) + (s.implicit ? 0 : 1) + 1;
    s.gc ^= 1;
    s.implicit = 0;
    s.f2_ready = 0;
    if (s.k < NS_HIST_F) P.res[s.sid].fnorm_hist[s.k] = fk;
    if (stop == NS_STOP_NONE && probe) {
      const double f2 = sqrt(ls_sum_parts(P, q, s.n, ls_probe_off(P.ldw)));
      s.mmm += 1;
      s.f2_ready = 1;
      if (f2 <= 0.25 * fk) stop = NS_STOP_FLOOR;
    }
    if (stop == NS_STOP_NONE && s.k >= P.k_max) stop = NS_STOP_K_MAX;
    s.ns_stop = stop;
    s.active = stop == NS_STOP_NONE;
    s.probe = 0;
    s.fk = fk;
    s.fprev = fk;
    P.ls[q] = s;
  }
}

// Refinement and report of each system whose Newton-Schulz phase ended;
// systems still iterating go to the overflow queue.
__global__ void __launch_bounds__(kLsNW * 64) ls_finish_kernel(BatchArgs P) {
  constexpr int NW = kLsNW;
  __shared__ double red[NW];
  const int nsys = ls_count(P);
  for (int q = blockIdx.x; q < nsys; q += gridDim.x) {
    const LsState s = P.ls[q];
    if (s.ns_stop == NS_STOP_NONE) {
      if (threadIdx.x == 0) {
        const int idx = atomicAdd(P.counter + 7, 1);
        P.ovf[idx] = s.sid + 1;
      }
      continue;
    }
    const BatchDesc d = P.desc[s.sid];
    const SlotMats sm = slot_mats<double>(P, ls_slot(P, q), nullptr);
    Ctl c;
    c.alpha = s.alpha;
    c.rel_resid = NAN;
    c.mmm = s.mmm;
    c.ns_steps = s.k;
    c.ns_stop = s.ns_stop;
    c.refine_steps = 0;
    c.refine_stop = NS_STOP_NONE;
    c.n_fnorm = (s.k + 1 < NS_HIST_F) ? s.k + 1 : NS_HIST_F;
    c.precision = NS_PREC_FP64;
    bool ok = false;
    if (s.ns_stop == NS_STOP_DIVERGED) {
      c.refine_stop = NS_STOP_DIVERGED;
    } else {
      ok = wg_refine<double, NW, NSR_BATCH_GR>(P, s.n, d.A, d.lda, d.b, d.theta,
                                               (const double*)(s.gc ? sm.G[1] : sm.G[0]), P.ldw,
                                               s.alpha, sm.r,
                                               s.bnorm, red, c);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      BatchResult* R = &P.res[s.sid];
      write_result(P, s.sid, true, true, ok, c, R->fnorm_hist, s.t_begin);
    }
    __syncthreads();
  }
}

template <typename T, int NW>
__global__ void __launch_bounds__(NW * 64) small_kernel(BatchArgs P) {
  constexpr bool dbl = sizeof(T) == 8;
  constexpr int LD = SmallLd<T>::value;
  __shared__ double red[NW];
  __shared__ double hist[NS_HIST_F];
  __shared__ double vec[4 * SMALL_N];
  __shared__ double part[NW * SMALL_N];
  __shared__ double a64[dbl ? 1 : SMALL_N * SMALL_N];
  __shared__ int s_idx;
  __shared__ __attribute__((aligned(16))) T mats[4 * SMALL_N * LD];
  const bool from_queue = dbl && !P.fp64_only;
  int* counter = P.counter + (from_queue ? 1 : 0);
  const int total = from_queue ? P.counter[2] : P.count;
  for (;;) {
    if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
    __syncthreads();
    const int q = s_idx;
    __syncthreads();
    if (q >= total) break;
    const int sid = from_queue ? P.retry[q] - 1 : P.order[q];
    const BatchDesc d = P.desc[sid];
    const int64_t t_begin = wall_clock64();
    Ctl c;
    const bool ok = wg_solve_small<T, NW>(P, d, mats, vec, a64, part, red, hist, c);
    __syncthreads();  // hist complete
    if (threadIdx.x == 0) write_result(P, sid, dbl, from_queue, ok, c, hist, t_begin);
    __syncthreads();
  }
}

}  // namespace

size_t batch_slot_bytes(int ldw) {
  const size_t nn = (size_t)ldw * ldw;
  // per-block partial sums: the team products' 32 x 32 blocks, or the
  // lockstep residual and probe products' 128 x 64 blocks
  const size_t team = ((size_t)ldw / 32) * ((size_t)ldw / 32);
  const size_t ls = 2 * (((size_t)ldw + Block<kLsGemmNW>::BM - 1) / Block<kLsGemmNW>::BM) *
                   (((size_t)ldw + Block<kLsGemmNW>::BN - 1) / Block<kLsGemmNW>::BN);
  const size_t blocks = team > ls ? team : ls;
  size_t b = 8 * nn * sizeof(float) + 7 * nn * sizeof(double) + 2 * (size_t)ldw * sizeof(double) +
             blocks * sizeof(double);
  return (b + 255) / 256 * 256;
}

template <typename T>
int launch_pass(const BatchArgs& a, int grid, int waves, hipStream_t st) {
  switch (waves) {
    case 1: hipLaunchKernelGGL((batch_kernel<T, 1>), dim3(grid), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((batch_kernel<T, 2>), dim3(grid), dim3(128), 0, st, a); break;
    case 4: hipLaunchKernelGGL((batch_kernel<T, 4>), dim3(grid), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL((batch_kernel<T, 8>), dim3(grid), dim3(512), 0, st, a); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename T>
int launch_small(const BatchArgs& a, int grid, int waves, hipStream_t st) {
  if (waves >= 8)
    hipLaunchKernelGGL((small_kernel<T, 8>), dim3(grid), dim3(512), 0, st, a);
  else
    hipLaunchKernelGGL((small_kernel<T, 4>), dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

bool small_fits(int max_n, int order) { return max_n <= SMALL_N && (order == 2 || order == 4); }

// Zero n 32-bit words (a kernel, not hipMemsetAsync: submissions may be
// captured into a HIP graph, where memset nodes are avoided).
__global__ void __launch_bounds__(256) zero_words_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0u;
}

int zero_words(void* p, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Float32 attempts with float64 escalation in one persistent launch
// (escalate_kernel), or the float64 pass alone.  With small = true every pass
// runs the LDS-resident kernel (four or eight waves): the float32 pass, then
// a float64 pass over its queue on wider workgroups (waves64), one per CU.
int launch_batch(const BatchArgs& a, int grid, int waves, int grid64, int waves64, bool small,
                 hipStream_t st) {
  if (small) {
    if (!a.fp64_only) {
      if (launch_small<float>(a, grid, waves, st)) return -1;
      if (!a.escalate) return 0;
      return launch_small<double>(a, grid64, waves64, st);
    }
    return launch_small<double>(a, grid, waves, st);
  }
  if (!a.fp64_only) {
    if (launch_pass<float>(a, grid, waves, st)) return -1;
    if (!a.escalate) return 0;
    return launch_pass<double>(a, grid64, waves64, st);
  }
  return launch_pass<double>(a, grid, waves, st);
}

// Float32 attempts with float64 escalation on two streams: the float32 pass
// on `st`, and beside it, on `side` (after ev_start, recorded on `st` once the
// submission's state is reset), the float64 team kernel (team_grid
// workgroups of four waves, slots after the float32 pass's).  Then, on `st`
// after both, a float64 pass re-solves whatever the team kernel left
// unclaimed (nothing, unless its workgroups ran out of waiting).
int launch_escalating(BatchArgs a, int grid, int waves, int team_grid, int grid64,
                      hipStream_t st, hipStream_t side, hipEvent_t ev_start,
                      hipEvent_t ev_side) {
  if (team_grid > 0) {
    if (hipEventRecord(ev_start, st) != hipSuccess || hipStreamWaitEvent(side, ev_start, 0) != hipSuccess)
      return -1;
    BatchArgs t = a;
    t.slot_base = grid;
    hipLaunchKernelGGL((team_kernel<4>), dim3(team_grid), dim3(256), 0, side, t);
    if (hipGetLastError() != hipSuccess) return -1;
  }
  switch (waves) {
    case 1: hipLaunchKernelGGL((f32_pass_kernel<1>), dim3(grid), dim3(64), 0, st, a); break;
    case 2: hipLaunchKernelGGL((f32_pass_kernel<2>), dim3(grid), dim3(128), 0, st, a); break;
    case 4: hipLaunchKernelGGL((f32_pass_kernel<4>), dim3(grid), dim3(256), 0, st, a); break;
    case 8: hipLaunchKernelGGL((f32_pass_kernel<8>), dim3(grid), dim3(512), 0, st, a); break;
    default: return -1;
  }
  if (hipGetLastError() != hipSuccess) return -1;
  if (team_grid > 0 && (hipEventRecord(ev_side, side) != hipSuccess ||
                        hipStreamWaitEvent(st, ev_side, 0) != hipSuccess))
    return -1;
  return launch_pass<double>(a, grid64, 8, st);
}

// Lockstep float64 re-solve of the float32 pass's queue (see the lockstep
// kernels), then the one-workgroup float64 pass over its overflow queue.
// The number of queued systems is known only on the device, so every launch
// is sized for the largest queue and does nothing for absent or finished
// systems.
int launch_lockstep(BatchArgs a, int sys_grid, int grid64, int cus, hipStream_t st) {
  a.ls_on = 1;
  int sexp = 0;
  while ((1 << sexp) < a.ns_order) ++sexp;
  constexpr int BM = Block<kLsGemmNW>::BM, BN = Block<kLsGemmNW>::BN;
  const int per = ((a.ldw + BM - 1) / BM) * ((a.ldw + BN - 1) / BN);
  const int nsys = std::min(a.count, a.ls_slots);
  const int ggrid = std::max(1, std::min(nsys * per + nsys, (16 / kLsGemmNW) * cus));
  const dim3 gblk(kLsGemmNW * 64);
  const int cgrid = std::max(1, (nsys + 63) / 64);
  sys_grid = std::max(1, sys_grid);
  const dim3 blk(kLsNW * 64);
  // Steps enqueued: enough for the stop rule to end every iteration of
  // kappa up to ~1e12 (28 steps of order 4); a system still iterating after
  // them is re-solved by the one-workgroup pass.
  const int steps = std::min(a.k_max, std::max(1, (2 * kLsSteps) / std::max(sexp, 1)));
  hipLaunchKernelGGL(ls_init_kernel, dim3(sys_grid), blk, 0, st, a);
  for (int k = 0; k < steps; ++k) {
    for (int i = 1; i < sexp; ++i) {
      hipLaunchKernelGGL(ls_gemm_kernel, dim3(ggrid), gblk, 0, st, a, (int)kLsPow, i);
      hipLaunchKernelGGL(ls_gemm_kernel, dim3(ggrid), gblk, 0, st, a, (int)kLsAsm, i);
    }
    hipLaunchKernelGGL(ls_gemm_kernel, dim3(ggrid), gblk, 0, st, a, (int)kLsGside, 0);
    hipLaunchKernelGGL(ls_gemm_kernel, dim3(ggrid), gblk, 0, st, a, (int)kLsResid, 0);
    hipLaunchKernelGGL(ls_gemm_kernel, dim3(ggrid), gblk, 0, st, a, (int)kLsProbe, 0);
    hipLaunchKernelGGL(ls_ctl_kernel, dim3(cgrid), dim3(64), 0, st, a);
  }
  hipLaunchKernelGGL(ls_finish_kernel, dim3(sys_grid), blk, 0, st, a);
  if (hipGetLastError() != hipSuccess) return -1;
  return launch_pass<double>(a, grid64, 8, st);
}

}  // namespace nsr

// ---------------------------------------------------------------------------
// Host side: the ns_batch_* entry points of include/nsr.h.
// ---------------------------------------------------------------------------

using namespace nsr;

namespace {

int bfail(int code, const char* msg) {
  ns_set_error(msg);
  return code;
}

constexpr size_t kBAlign = 256;
inline size_t balign(size_t x) { return (x + kBAlign - 1) / kBAlign * kBAlign; }
inline int ldw_for(int64_t max_n) { return (int)((max_n + 31) / 32 * 32); }

size_t batch_layout(int64_t max_n, int max_count, int slots) {
  size_t b = 0;
  b += balign((size_t)max_count * sizeof(BatchDesc));
  b += balign((size_t)max_count * sizeof(BatchResult));
  b += balign((size_t)max_count * sizeof(int32_t));   // order
  b += balign((size_t)max_count * sizeof(int32_t));   // float64 queue
  b += balign(kCounters * sizeof(int32_t));           // counters
  b += balign((size_t)max_count * sizeof(TeamState)); // float64 teams
  b += balign((size_t)max_count * sizeof(LsState));   // lockstep states
  b += balign((size_t)max_count * sizeof(int32_t));   // overflow queue
  b += (size_t)slots * batch_slot_bytes(ldw_for(max_n));
  return b;
}

}  // namespace

struct ns_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t max_n = 0;
  int max_count = 0;
  int slots = 0;
  int ldw = 0;
  int precision = NS_PREC_FP32;
  int waves = 4;
  int ls_min_count = kLsMinCount;   // lockstep float64 re-solve from this many systems (0: off)
  int groups = 0;  // launch size (<= slots); 0: all slots
  int cus = 256;   // compute units of the device
  int64_t ticks_ms = 100000;   // device wall-clock ticks per millisecond
  BatchDesc* d_desc = nullptr;
  BatchResult* d_res = nullptr;
  int32_t* d_order = nullptr;
  int32_t* d_counter = nullptr;   // kCounters counters (see BatchArgs)
  int32_t* d_retry = nullptr;
  TeamState* d_team = nullptr;
  LsState* d_ls = nullptr;       // lockstep states (max_count)
  int32_t* d_ovf = nullptr;      // overflow queue (max_count)
  char* d_slots = nullptr;
  hipEvent_t done = nullptr;
  hipStream_t side = nullptr;     // the float64 team kernel's stream
  hipEvent_t ev_start = nullptr, ev_side = nullptr;
  uint64_t next_ticket = 0;
  uint64_t inflight = 0;
  int inflight_count = 0;
  bool busy = false;
  uint64_t last_polled = 0;   // ticket whose results h_res holds
  bool have_results = false;
  std::vector<BatchDesc> h_desc;
  std::vector<int32_t> h_order;
  std::vector<BatchResult> h_res;
  hipGraphExec_t gexec = nullptr;  // the captured submission (opts->graph)
  hipStream_t cap = nullptr;        // private stream for the capture
  std::vector<char> graph_key;      // what gexec was captured for (empty: none)
  ns_ledger* ledger = nullptr;   // HBM admission (ns_batch_set_ledger), may be NULL
  size_t held = 0;               // bytes the in-flight submission holds in it
};

namespace {

// The float64 team kernel beside the float32 pass is switched off: its first
// GPU run stalled (every wait of the team kernel polled with acquire loads,
// and each poll invalidated the L2 of its XCD under the float32 pass; fixed),
// and the run that tested the fix stalled again, in a batch with nine team
// workgroups (one team workgroup had passed), with no cause found.  Escalating
// submissions run the float32 pass and then the float64 pass over its queue.
constexpr bool kTeamKernelEnabled = false;

// A submission's launch: its arguments and grid, decided on the host.
struct Launch {
  BatchArgs a;
  int grid, grid64;
  int max_n;
  bool small;
};

// Checks and host-side set-up of a submission (descriptors in largest-first
// order, launch arguments); no device work.
int batch_prepare(ns_batch* B, int count, const int64_t* n, const double* const* A,
                  const int64_t* lda, const double* const* b, double* const* theta,
                  const ns_solve_opts* o, Launch& L) {
  if (count < 0) return bfail(NS_EINVAL, "count < 0");
  if (count > B->max_count) return bfail(NS_ENOMEM, "count exceeds the batch capacity");
  if (!o) return bfail(NS_EINVAL, "null opts");
  if (o->factorization != NS_FACT_SQUARING)
    return bfail(NS_EINVAL, "batched solves use the squaring form");
  if (o->order < 2 || (o->order & (o->order - 1)) != 0)
    return bfail(NS_EINVAL, "order must be 2^s >= 2");
  if (o->k_max < 1 || o->k_max > NS_HIST_F - 1) return bfail(NS_EINVAL, "k_max must be in 1..64");
  if (o->refine_max < 0) return bfail(NS_EINVAL, "refine_max < 0");
  if (o->scale != NS_SCALE_FROBENIUS && o->scale != NS_SCALE_INF_HALF &&
      o->scale != NS_SCALE_DIAG)
    return bfail(NS_EINVAL, "unknown scale");
  if (o->scale == NS_SCALE_INF_HALF && !(o->eps >= 0.0)) return bfail(NS_EINVAL, "eps < 0");
  if (o->theta0_mode != 0) return bfail(NS_EINVAL, "batched solves start from theta_0 = b/alpha");
  if (count > 0 && (!n || !A || !lda || !b || !theta)) return bfail(NS_EINVAL, "null array");
  B->h_desc.resize(count);
  B->h_order.resize(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1) return bfail(NS_EINVAL, "system size < 1");
    if (n[i] > B->max_n) return bfail(NS_ENOMEM, "system larger than the batch's max_n");
    if (lda[i] < n[i]) return bfail(NS_EINVAL, "lda < n");
    if (!A[i] || !b[i] || !theta[i]) return bfail(NS_EINVAL, "null system pointer");
    B->h_desc[i] = BatchDesc{A[i], b[i], theta[i], lda[i], (int32_t)n[i], 0};
    B->h_order[i] = i;
  }
  // Largest systems first (longest-processing-time order for the work pull).
  std::stable_sort(B->h_order.begin(), B->h_order.end(),
                   [&](int32_t x, int32_t y) { return B->h_desc[x].n > B->h_desc[y].n; });
  BatchArgs& a = L.a;
  a = BatchArgs{};
  a.desc = B->d_desc;
  a.res = B->d_res;
  a.order = B->d_order;
  a.counter = B->d_counter;
  a.retry = B->d_retry;
  a.team = B->d_team;
  a.ls = B->d_ls;
  a.ovf = B->d_ovf;
  a.ls_slots = B->slots;
  a.ls_on = 0;
  a.ticks_ms = B->ticks_ms;
  a.slots = B->d_slots;
  a.slot_bytes = (int64_t)batch_slot_bytes(B->ldw);
  a.count = count;
  a.ldw = B->ldw;
  a.ns_order = o->order;
  a.k_max = o->k_max;
  a.refine_max = o->refine_max;
  a.floor_detect = o->floor_detect;
  a.escalate = (B->precision == NS_PREC_FP32) ? 1 : 0;
  a.fp64_only = (B->precision == NS_PREC_FP64) ? 1 : 0;
  a.scale = o->scale;
  a.eps = o->eps;
  a.f_tol = o->f_tol;
  a.resid_tol = o->resid_tol;
  L.grid = B->groups > 0 ? B->groups : B->slots;
  if (L.grid > B->slots) L.grid = B->slots;
  if (L.grid > count) L.grid = count;
  L.grid64 = B->cus < B->slots ? B->cus : B->slots;
  if (L.grid64 > count) L.grid64 = count;
  int max_sys = 0;
  for (int i = 0; i < count; ++i) max_sys = std::max(max_sys, (int)n[i]);
  L.small = small_fits(max_sys, o->order);
  L.max_n = max_sys;
  return NS_OK;
}

// Upload of the prepared descriptors (host vectors of the handle) on st.
int batch_upload(ns_batch* B, int count, hipStream_t st) {
  if (hipSetDevice(B->device) != hipSuccess) return bfail(NS_EHIP, "hipSetDevice failed");
  if (count > 0 &&
      (hipMemcpyAsync(B->d_desc, B->h_desc.data(), count * sizeof(BatchDesc),
                      hipMemcpyHostToDevice, st) != hipSuccess ||
       hipMemcpyAsync(B->d_order, B->h_order.data(), count * sizeof(int32_t),
                      hipMemcpyHostToDevice, st) != hipSuccess))
    return bfail(NS_EHIP, "descriptor upload failed");
  return NS_OK;
}

// The submission's device work after the upload: reset of its counters,
// queue and team states, then the persistent kernels.  Enqueued on st (the
// handle's stream, or a stream under graph capture).
int batch_launch(ns_batch* B, const Launch& L, hipStream_t st, bool allow_team) {
  const int count = L.a.count;
  if (zero_words(B->d_counter, kCounters * sizeof(int32_t), st) ||
      zero_words(B->d_retry, (size_t)count * sizeof(int32_t), st) ||
      zero_words(B->d_team, (size_t)count * sizeof(TeamState), st))
    return bfail(NS_EHIP, "counter reset failed");
  if (allow_team && kTeamKernelEnabled && L.grid > 0 && !L.small && L.a.escalate) {
    // the team kernel: one workgroup per CU, in the slots after the float32
    // pass's (none when the slots are all taken)
    int team_grid = std::min(B->cus, B->slots - L.grid);
    if (team_grid < 0) team_grid = 0;
    if (launch_escalating(L.a, L.grid, B->waves, team_grid, L.grid64, st, B->side, B->ev_start,
                          B->ev_side) != 0)
      return bfail(NS_EHIP, "batch kernel launch failed");
    return NS_OK;
  }
  const bool lockstep = NSR_BATCH_LOCKSTEP && !L.small && L.a.escalate && L.max_n >= kLsMinN &&
                        B->ls_min_count > 0 && L.a.count >= B->ls_min_count;
  if (L.grid > 0 && lockstep) {
    if (launch_pass<float>(L.a, L.grid, B->waves, st) != 0 ||
        launch_lockstep(L.a, std::min(L.a.count, 2 * B->cus), L.grid64, B->cus, st) != 0)
      return bfail(NS_EHIP, "batch kernel launch failed");
    return NS_OK;
  }
  if (L.grid > 0 && launch_batch(L.a, L.grid, B->waves, L.grid64, 8, L.small, st) != 0)
    return bfail(NS_EHIP, "batch kernel launch failed");
  return NS_OK;
}

int batch_enqueue(ns_batch* B, int count, const int64_t* n, const double* const* A,
                  const int64_t* lda, const double* const* b, double* const* theta,
                  const ns_solve_opts* o) {
  Launch L;
  if (int rc = batch_prepare(B, count, n, A, lda, b, theta, o, L)) return rc;
  B->graph_key.clear();   // the device descriptors change: a captured graph is stale
  if (int rc = batch_upload(B, count, B->stream)) return rc;
  return batch_launch(B, L, B->stream, true);
}

// Key of a submission for graph reuse: every input the captured work
// depends on (launch shape, options, descriptors).
std::vector<char> graph_key(const ns_batch* B, const Launch& L, const ns_solve_opts* o) {
  std::vector<char> k;
  auto put = [&](const void* p, size_t n) {
    const char* c = static_cast<const char*>(p);
    k.insert(k.end(), c, c + n);
  };
  put(&B->waves, sizeof(B->waves));
  put(&B->groups, sizeof(B->groups));
  put(&L.grid, sizeof(L.grid));
  put(&L.grid64, sizeof(L.grid64));
  ns_solve_opts oc = *o;
  oc.graph = 0;
  put(&oc, sizeof(oc));
  put(B->h_desc.data(), B->h_desc.size() * sizeof(BatchDesc));
  return k;
}

// Graph path of ns_batch_submit: replay the captured submission when this
// one is identical to it, else upload, capture the device work on a private
// stream, instantiate, and launch the graph on the handle's stream.
int batch_enqueue_graph(ns_batch* B, int count, const int64_t* n, const double* const* A,
                        const int64_t* lda, const double* const* b, double* const* theta,
                        const ns_solve_opts* o) {
  Launch L;
  if (int rc = batch_prepare(B, count, n, A, lda, b, theta, o, L)) return rc;
  if (hipSetDevice(B->device) != hipSuccess) return bfail(NS_EHIP, "hipSetDevice failed");
  std::vector<char> key = graph_key(B, L, o);
  if (!B->gexec || key != B->graph_key) {
    B->graph_key.clear();
    if (B->gexec) {
      (void)hipGraphExecDestroy(B->gexec);
      B->gexec = nullptr;
    }
    if (int rc = batch_upload(B, count, B->stream)) return rc;
    if (hipStreamSynchronize(B->stream) != hipSuccess) return bfail(NS_EHIP, "stream sync failed");
    if (!B->cap && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
      return bfail(NS_EHIP, "hipStreamCreate failed");
    if (hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bfail(NS_EHIP, "hipStreamBeginCapture failed");
    const int rc = batch_launch(B, L, B->cap, false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(B->cap, &g);
    if (rc != NS_OK || e != hipSuccess || !g) {
      if (g) (void)hipGraphDestroy(g);
      return rc != NS_OK ? rc : bfail(NS_EHIP, "hipStreamEndCapture failed");
    }
    const hipError_t ei = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      B->gexec = nullptr;
      return bfail(NS_EHIP, "hipGraphInstantiate failed");
    }
    B->graph_key = std::move(key);
  }
  if (hipGraphLaunch(B->gexec, B->stream) != hipSuccess) return bfail(NS_EHIP, "hipGraphLaunch failed");
  return NS_OK;
}

}  // namespace

extern "C" {

size_t ns_batch_workspace_bytes(int64_t max_n, int max_count, int slots) {
  if (max_n < 1 || max_count < 1 || slots < 1) return 0;
  return batch_layout(max_n, max_count, slots);
}

int ns_batch_create(int device, void* hip_stream, int64_t max_n, int max_count, int slots,
                    int precision, void* workspace, size_t bytes, ns_batch** out) {
  if (!out) return bfail(NS_EINVAL, "null out");
  *out = nullptr;
  if (max_n < 1 || max_n > 4096) return bfail(NS_EINVAL, "max_n must be in 1..4096");
  if (max_count < 1 || slots < 1) return bfail(NS_EINVAL, "max_count and slots must be >= 1");
  if (precision != NS_PREC_FP32 && precision != NS_PREC_FP64)
    return bfail(NS_EINVAL, "batched precision must be NS_PREC_FP32 or NS_PREC_FP64");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kBAlign) != 0)
    return bfail(NS_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (bytes < batch_layout(max_n, max_count, slots)) return bfail(NS_ENOMEM, "workspace too small");
  if (hipSetDevice(device) != hipSuccess) return bfail(NS_EHIP, "hipSetDevice failed");
  ns_batch* B = new (std::nothrow) ns_batch();
  if (!B) return bfail(NS_ENOMEM, "host allocation failed");
  B->device = device;
  B->stream = reinterpret_cast<hipStream_t>(hip_stream);
  B->max_n = max_n;
  B->max_count = max_count;
  B->slots = slots;
  B->ldw = ldw_for(max_n);
  B->precision = precision;
  {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        v > 0)
      B->cus = v;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess &&
        khz > 0)
      B->ticks_ms = khz;
  }
  char* p = reinterpret_cast<char*>(workspace);
  B->d_desc = reinterpret_cast<BatchDesc*>(p);
  p += balign((size_t)max_count * sizeof(BatchDesc));
  B->d_res = reinterpret_cast<BatchResult*>(p);
  p += balign((size_t)max_count * sizeof(BatchResult));
  B->d_order = reinterpret_cast<int32_t*>(p);
  p += balign((size_t)max_count * sizeof(int32_t));
  B->d_retry = reinterpret_cast<int32_t*>(p);
  p += balign((size_t)max_count * sizeof(int32_t));
  B->d_counter = reinterpret_cast<int32_t*>(p);
  p += balign(kCounters * sizeof(int32_t));
  B->d_team = reinterpret_cast<TeamState*>(p);
  p += balign((size_t)max_count * sizeof(TeamState));
  B->d_ls = reinterpret_cast<LsState*>(p);
  p += balign((size_t)max_count * sizeof(LsState));
  B->d_ovf = reinterpret_cast<int32_t*>(p);
  p += balign((size_t)max_count * sizeof(int32_t));
  B->d_slots = p;
  if (hipEventCreate(&B->done) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_start, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_side, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&B->side, hipStreamNonBlocking) != hipSuccess) {
    if (B->done) (void)hipEventDestroy(B->done);
    if (B->ev_start) (void)hipEventDestroy(B->ev_start);
    if (B->ev_side) (void)hipEventDestroy(B->ev_side);
    delete B;
    return bfail(NS_EHIP, "hipEventCreate / hipStreamCreate failed");
  }
  *out = B;
  return NS_OK;
}

int ns_batch_set_lockstep(ns_batch* B, int min_count) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (min_count < 0) return bfail(NS_EINVAL, "min_count < 0");
  B->ls_min_count = min_count;
  B->graph_key.clear();
  return NS_OK;
}

int ns_batch_set_launch(ns_batch* B, int waves_per_group, int groups) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4 &&
      waves_per_group != 8)
    return bfail(NS_EINVAL, "waves_per_group must be 1, 2, 4 or 8");
  if (groups < 0 || groups > B->slots) return bfail(NS_EINVAL, "groups must be in 0..slots");
  B->waves = waves_per_group;
  B->groups = groups;
  return NS_OK;
}

int ns_batch_set_ledger(ns_batch* B, ns_ledger* ledger) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (B->busy) return bfail(NS_EBUSY, "a submission is still in flight; poll it first");
  B->ledger = ledger;
  return NS_OK;
}

int ns_batch_submit(ns_batch* B, int count, const int64_t* n, const double* const* A,
                    const int64_t* lda, const double* const* b, double* const* theta,
                    const ns_solve_opts* opts, uint64_t* ticket) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (B->busy) return bfail(NS_EBUSY, "a submission is still in flight; poll it first");
  size_t bytes = 0;
  if (B->ledger) {
    // Admission by HBM footprint: the submission's A, b and theta.
    if (count > 0 && !n) return bfail(NS_EINVAL, "null array");
    for (int i = 0; i < count; ++i)
      if (n[i] > 0) bytes += ((size_t)n[i] * (size_t)n[i] + 2 * (size_t)n[i]) * sizeof(double);
    const int rc = ns_ledger_admit(B->ledger, bytes);
    if (rc != NS_OK) return rc;
  }
  const int rc_enq = (opts && opts->graph)
                        ? batch_enqueue_graph(B, count, n, A, lda, b, theta, opts)
                        : batch_enqueue(B, count, n, A, lda, b, theta, opts);
  if (rc_enq != NS_OK) {
    if (B->ledger) (void)ns_ledger_release(B->ledger, bytes);
    return rc_enq;
  }
  if (hipEventRecord(B->done, B->stream) != hipSuccess) {
    (void)hipStreamSynchronize(B->stream);
    if (B->ledger) (void)ns_ledger_release(B->ledger, bytes);
    return bfail(NS_EHIP, "hipEventRecord failed");
  }
  B->held = bytes;
  B->busy = true;
  B->inflight = ++B->next_ticket;
  B->inflight_count = count;
  if (ticket) *ticket = B->inflight;
  return NS_OK;
}

int ns_batch_timeline(ns_batch* B, uint64_t ticket, double* times_us, int32_t* workgroup) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (!B->have_results || ticket != B->last_polled)
    return bfail(NS_EINVAL, "timeline of a ticket that was not the last one polled");
  if (!times_us) return bfail(NS_EINVAL, "null times_us");
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, B->device) != hipSuccess ||
      khz <= 0)
    return bfail(NS_EHIP, "wall clock rate unavailable");
  const double us_per_tick = 1e3 / (double)khz;
  int64_t t0 = INT64_MAX;
  for (const BatchResult& r : B->h_res)
    for (int j = 0; j < 4; j += 2)
      if (r.clock[j] != 0 && r.clock[j] < t0) t0 = r.clock[j];
  for (size_t i = 0; i < B->h_res.size(); ++i) {
    const BatchResult& r = B->h_res[i];
    for (int j = 0; j < 4; ++j) {
      const bool ran = r.clock[j & ~1] != 0;
      times_us[4 * i + j] = ran ? (double)(r.clock[j] - t0) * us_per_tick : NAN;
    }
    if (workgroup) {
      workgroup[2 * i] = r.wg[0];
      workgroup[2 * i + 1] = r.wg[1];
    }
  }
  return NS_OK;
}

int ns_batch_poll(ns_batch* B, uint64_t ticket, int wait, ns_solve_report* reports) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (!B->busy || ticket != B->inflight) return bfail(NS_EINVAL, "unknown ticket");
  if (wait) {
    if (hipEventSynchronize(B->done) != hipSuccess) return bfail(NS_EHIP, "hipEventSynchronize failed");
  } else {
    hipError_t q = hipEventQuery(B->done);
    if (q == hipErrorNotReady) return NS_EBUSY;
    if (q != hipSuccess) return bfail(NS_EHIP, "hipEventQuery failed");
  }
  const int cnt = B->inflight_count;
  B->h_res.resize(cnt);
  int32_t hc[kCounters] = {};
  if (cnt > 0 && (hipMemcpy(B->h_res.data(), B->d_res, cnt * sizeof(BatchResult),
                            hipMemcpyDeviceToHost) != hipSuccess ||
                  hipMemcpy(hc, B->d_counter, sizeof(hc), hipMemcpyDeviceToHost) != hipSuccess))
    return bfail(NS_EHIP, "result download failed");
  B->busy = false;
  if (B->ledger && B->held) (void)ns_ledger_release(B->ledger, B->held);
  if (hc[5] != 0) {
    // A bounded wait of the escalating kernel ran out (a team's blocks or a
    // queue entry never arrived): the results cannot be trusted.
    B->have_results = false;
    return bfail(NS_EHIP, hc[5] == 1 ? "a float64 team product timed out"
                                     : "a float64 queue entry timed out");
  }
  B->held = 0;
  B->last_polled = ticket;
  B->have_results = true;
  int worst = NS_OK;
  for (int i = 0; i < cnt; ++i) {
    const BatchResult& r = B->h_res[i];
    if (r.status != NS_OK && worst == NS_OK) worst = r.status;
    if (!reports) continue;
    ns_solve_report& R = reports[i];
    memset(&R, 0, sizeof(R));
    R.status = r.status;
    R.ns_stop = r.ns_stop;
    R.refine_stop = r.refine_stop;
    R.ns_steps = r.ns_steps;
    R.refine_steps = r.refine_steps;
    R.precision = r.precision;
    R.alpha = r.alpha;
    R.rel_resid = r.rel_resid;
    R.mmm = r.mmm;
    const double nn = (double)B->h_desc[i].n;
    R.gemm_flop = 2.0 * nn * nn * nn * (double)r.mmm;
    R.n_fnorm = r.n_fnorm;
    for (int j = 0; j < r.n_fnorm && j < NS_HIST_F; ++j) R.fnorm_hist[j] = r.fnorm_hist[j];
    R.n_resid = 0;
  }
  return worst == NS_OK ? NS_OK : NS_ENOCONV;
}

int ns_batch_autotune(ns_batch* B, int count, const int64_t* n, const double* const* A,
                      const int64_t* lda, const double* const* b, double* const* theta,
                      const ns_solve_opts* opts, int* best_waves, int* best_groups,
                      double* best_ms) {
  if (!B) return bfail(NS_EINVAL, "null batch");
  if (B->busy) return bfail(NS_EBUSY, "a submission is still in flight; poll it first");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return bfail(NS_EHIP, "hipEventCreate failed");
  int bw = 4, bg = 0;
  float bms = 1e30f;
  const int waves_c[4] = {1, 2, 4, 8};
  const int cus = B->cus;
  const int per_cu_c[4] = {1, 2, 4, 8};
  int rc = NS_OK;
  for (int wi = 0; wi < 4 && rc == NS_OK; ++wi) {
    int prev_groups = -1;
    for (int gi = 0; gi < 4 && rc == NS_OK; ++gi) {
      int groups = per_cu_c[gi] * cus;
      if (groups > B->slots) groups = B->slots;
      if (groups == prev_groups) continue;
      prev_groups = groups;
      B->waves = waves_c[wi];
      B->groups = groups;
      if (hipEventRecord(e0, B->stream) != hipSuccess) { rc = bfail(NS_EHIP, "event"); break; }
      rc = batch_enqueue(B, count, n, A, lda, b, theta, opts);
      if (rc) break;
      if (hipEventRecord(e1, B->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = bfail(NS_EHIP, "event");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < bms) {
        bms = ms;
        bw = waves_c[wi];
        bg = groups;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  B->waves = bw;
  B->groups = bg;
  if (best_waves) *best_waves = bw;
  if (best_groups) *best_groups = bg;
  if (best_ms) *best_ms = bms;
  return NS_OK;
}

int ns_batch_destroy(ns_batch* B) {
  if (!B) return NS_OK;
  if (B->busy) (void)hipEventSynchronize(B->done);
  if (B->busy && B->ledger && B->held) (void)ns_ledger_release(B->ledger, B->held);
  if (B->side) (void)hipStreamSynchronize(B->side);
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  if (B->done) (void)hipEventDestroy(B->done);
  if (B->ev_start) (void)hipEventDestroy(B->ev_start);
  if (B->ev_side) (void)hipEventDestroy(B->ev_side);
  if (B->side) (void)hipStreamDestroy(B->side);
  delete B;
  return NS_OK;
}

}  // extern "C"
