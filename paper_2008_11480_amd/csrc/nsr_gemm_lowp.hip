// Float32 and bf16 MFMA GEMMs for gfx950 with the solver's fused epilogue
//
//   D = diag * I + scale * (X op(Y)) + E1 + E2
//
// * gemm_f32_nn: X (m x k) and Y (k x n) row-major float32, float32
//   accumulate (v_mfma_f32_16x16x4_f32).  Used where rounding would be
//   amplified by the condition number: the residual F = I - A G, the G-side
//   update G + G C and the composite merge (float32 / mixed modes).
// * gemm_bf16_nt: X (m x k) and Y (n x k) row-major bf16, D = X Y^T, float32
//   accumulate (v_mfma_f32_32x32x16_bf16).  Used for the powers of F and the
//   identity-offset assembly of the mixed mode.  Those operands are
//   polynomials in F (symmetric in exact arithmetic), so Y^T = Y up to a
//   rounding asymmetry far below the bf16 rounding of the operands, and the
//   NT form lets both operands be read with K contiguous.
//
// * gemm_f16s_nt: the float32-class product of the split mode, D = X Y^T
//   from half-precision hi / lo planes of both operands (three fp16 MFMA
//   products, v_mfma_f32_32x32x16_f16), after absmax / split_rows /
//   split_trans have scaled and split the float32 operands.
// * gemm_bf16_sym / gemm_bf16_sym_fixup: a symmetric-output bf16 product
//   (upper tiles + mirror); switched off by the library (it faulted the GPU
//   on its first test, cause not found) and kept for a later fix.
//
// All write float32 D, optionally a bf16 copy Db (next GEMM's operand), and
// optionally one float64 partial sum of D^2 per tile.
//
// Accumulator layouts (gfx950, measured): for 16x16x4 f32, element r of lane
// l is D[4 (l/16) + r][l % 16]; for 32x32x16 bf16 it is
// D[8 (r/4) + 4 (l/32) + r % 4][l % 32], and the bf16 operand element e of
// lane l is K index 8 (l/32) + e.
//
// Tiling: large outputs take 256 x 256 workgroup tiles of eight waves whose
// K slabs go from global memory straight into a ring of LDS stages
// (global_load_lds_dwordx4), one workgroup per CU; smaller outputs take the
// float64 GEMM's scheme (128 x 128 or 64 x 64 tiles, 4 waves, K slabs staged
// global -> registers (one slab ahead) -> two LDS buffers, two workgroups per
// CU; the 128 x 128 tiles of every family take their slabs by LDS DMA too
// where the operands allow it).  Every kernel walks its tiles in an
// XCD-aware grouped order.
#include "nsr_internal.h"

#ifndef NSR_BF16_HUGE
#define NSR_BF16_HUGE 1
#endif
// 1: raise the wave's issue priority while it runs a slab's MFMAs.
#ifndef NSR_LP_SETPRIO
#define NSR_LP_SETPRIO 1
#endif
#ifndef NSR_BF16_HUGE_BK
#define NSR_BF16_HUGE_BK 64
#endif
// 1: 256 x 256 float32 tiles (LDS-DMA kernel) where its requirements hold.
#ifndef NSR_F32_DMA
#define NSR_F32_DMA 1
#endif
// 1: the 128 x 128 float32 and bf16 tiles take their K slabs by LDS DMA
// where the operands allow it (the split tiles follow NSR_F16S_DMA).
#ifndef NSR_F32_DMA128
#define NSR_F32_DMA128 1
#endif
#ifndef NSR_BF16_DMA128
#define NSR_BF16_DMA128 1
#endif
// 1: 256 x 256 split half-precision tiles use the LDS-DMA kernel where its
// requirements hold.
#ifndef NSR_F16S_DMA
#define NSR_F16S_DMA 1
#endif
// Fragments of addends the float32 LDS-DMA kernel's epilogue loads ahead.
#ifndef NSR_F32_EPI_PD
#define NSR_F32_EPI_PD 4
#endif
// Chunks of addends the bf16 LDS-DMA kernel's epilogue loads ahead.
#ifndef NSR_BF16_EPI_PD
#define NSR_BF16_EPI_PD 2
#endif
// 1: 256 x 256 bf16 tiles use the LDS-DMA kernel where its requirements hold.
#ifndef NSR_BF16_DMA
#define NSR_BF16_DMA 1
#endif

namespace nsr {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

namespace {

__device__ __forceinline__ void map_tile_lp(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int ntiles = tiles_m * tiles_n;
  int t = bid;
  if ((ntiles & 7) == 0) {
    const int per = ntiles >> 3;
    t = (bid & 7) * per + (bid >> 3);
  }
  constexpr int GM = 8;
  const int group_size = GM * tiles_n;
  const int g = t / group_size;
  const int first_m = g * GM;
  const int gm = min(tiles_m - first_m, GM);
  const int r = t - g * group_size;
  tm = first_m + r % gm;
  tn = r / gm;
}

// Shared epilogue of one output element; e1 / e2 are the addends E1, E2 at
// (row, col), loaded beforehand (0 where absent).
__device__ __forceinline__ void put(const GemmLpArgs& p, int64_t row, int64_t col, float acc,
                                    float e1, float e2, double& ss) {
  float v = p.scale * acc;
  if (row == col) v += p.diag;
  if (p.E1) v += e1;
  if (p.E2) v += e2;
  if (p.D) p.D[row * p.ldd + col] = v;
  if (p.Db) p.Db[row * p.lddb + col] = __builtin_bit_cast(uint16_t, (__bf16)v);
  ss += (double)v * (double)v;
}

// Addends of one accumulator fragment (R elements per lane at rows row_of(r),
// column col), loaded together ahead of the fragment's stores: loads and
// stores share one in-order completion counter, so a load issued after a
// store cannot complete before the store does, and loading per element after
// the previous element's store would put a memory round trip on every
// element.
template <int R, class RowOf>
__device__ __forceinline__ void load_addends(const GemmLpArgs& p, int64_t col, RowOf row_of,
                                             float (&e1)[R], float (&e2)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t row = row_of(r);
    const bool in = row < p.M && col < p.N;
    e1[r] = (p.E1 && in) ? p.E1[row * p.lde1 + col] : 0.0f;
    e2[r] = (p.E2 && in) ? p.E2[row * p.lde2 + col] : 0.0f;
  }
}

template <int NWAVES = 4>
__device__ __forceinline__ void write_partial(const GemmLpArgs& p, double ss, double* red,
                                              int tm, int tn, int tiles_n) {
  if (!p.partial) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) t += red[w];
    p.partial[(int64_t)tm * tiles_n + tn] = t;
  }
}

// ---------------------------------------------------------------------------
// float32, NN
// ---------------------------------------------------------------------------
// DMA form (128 x 128 tiles, BK = 32, two 32 KB stages; K a multiple of 32,
// N a multiple of 4, row strides multiples of 4 floats, 16-byte aligned X
// and Y): the K slabs go from global memory straight into LDS with
// global_load_lds_dwordx4, slab kt + 1 issued in two parts during slab kt's
// first two MFMA steps, one barrier per slab.  X rows (128 B) keep chunk c at
// c ^ ((row >> 1) & 7); Y rows (512 B) keep chunk c at c ^ 4 (k & 3), so the
// one-float-per-lane operand reads (16 rows or columns x 4 k) touch 64
// different banks.  The MFMA sequence and the accumulator layout are those of
// the register-staged loop (the results are the same bits) and the epilogue
// is shared.  Rows past M and columns past N of edge tiles read row M - 1
// and the last four columns and feed only outputs that are not stored.
template <int BM, int BN, int BK, bool VEC, bool DMA = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
gemm_f32_nn_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int NT = 256;
  constexpr int WTM = BM / 2, WTN = BN / 2;
  constexpr int FM = WTM / 16, FN = WTN / 16;
  // Row strides (floats).  An MFMA operand read has 16 lanes along one
  // dimension and 4 along K: X rows 36 floats apart put the 16 rows x 4 k in
  // 64 different banks; Y rows (k) must be 16 banks apart for the same
  // (BN + 4 put consecutive k rows 4 banks apart: 40% conflict cycles).
  constexpr int XS = BK + 4;
  constexpr int YS = BN + 16;
  constexpr int XV = (BM * BK / 4) / NT;  // float4 per thread
  constexpr int YV = (BK * BN / 4) / NT;
  static_assert(XV >= 1 && YV >= 1, "tile too small");
  static_assert(!DMA || (BM == 128 && BN == 128 && BK == 32 && VEC),
                "DMA form: 128 x 128 tiles, 32-deep slabs");
  // One LDS arena: the two register-staged slab buffers of X and Y, or the
  // DMA ring (two stages of BM x BK and BK x BN floats).
  constexpr int ARENA = 2 * BM * XS + 2 * BK * YS;
  static_assert(!DMA || ARENA >= 2 * (BM * BK + BK * BN), "DMA ring fits the arena");
  __shared__ __attribute__((aligned(1024))) float arena[ARENA];
  __shared__ double red[4];
  float (*Xs)[BM * XS] = reinterpret_cast<float (*)[BM * XS]>(arena);
  float (*Ys)[BK * YS] = reinterpret_cast<float (*)[BK * YS]>(arena + 2 * BM * XS);

  const float* X = static_cast<const float*>(p.X);
  const float* Y = static_cast<const float*>(p.Y);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  float4 xr[XV], yr[YV];

  // Interior tiles load full slabs with unchecked 16-byte loads (wave-uniform
  // branch); edge tiles and a partial last K slab take the checked path.
  const bool interior = VEC && (m0 + BM <= M) && (n0 + BN <= N);
  auto load = [&](int64_t k0) {
    if (interior && k0 + BK <= K) {
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int idx = tid + NT * v;
        xr[v] = *reinterpret_cast<const float4*>(X + (m0 + idx / (BK / 4)) * p.ldx + k0 +
                                                 (idx % (BK / 4)) * 4);
      }
#pragma unroll
      for (int v = 0; v < YV; ++v) {
        const int idx = tid + NT * v;
        yr[v] = *reinterpret_cast<const float4*>(Y + (k0 + idx / (BN / 4)) * p.ldy + n0 +
                                                 (idx % (BN / 4)) * 4);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
      const int64_t gm = m0 + row, gk = k0 + c;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gm < M) {
        const float* src = X + gm * p.ldx + gk;
        if (VEC && gk + 3 < K) {
          val = *reinterpret_cast<const float4*>(src);
        } else {
          if (gk < K) val.x = src[0];
          if (gk + 1 < K) val.y = src[1];
          if (gk + 2 < K) val.z = src[2];
          if (gk + 3 < K) val.w = src[3];
        }
      }
      xr[v] = val;
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
      const int64_t gk = k0 + row, gn = n0 + c;
      float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gk < K) {
        const float* src = Y + gk * p.ldy + gn;
        if (VEC && gn + 3 < N) {
          val = *reinterpret_cast<const float4*>(src);
        } else {
          if (gn < N) val.x = src[0];
          if (gn + 1 < N) val.y = src[1];
          if (gn + 2 < N) val.z = src[2];
          if (gn + 3 < N) val.w = src[3];
        }
      }
      yr[v] = val;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 4), c = (idx % (BK / 4)) * 4;
      *reinterpret_cast<float4*>(&Xs[buf][row * XS + c]) = xr[v];
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BN / 4), c = (idx % (BN / 4)) * 4;
      *reinterpret_cast<float4*>(&Ys[buf][row * YS + c]) = yr[v];
    }
  };

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int nk = (int)((K + BK - 1) / BK);
  const int lr = lane & 15, lk = lane >> 4;
  if constexpr (DMA) {
    constexpr int XB = BM * BK * 4, SB = XB + BK * BN * 4;   // 16 KB of X, 16 KB of Y
    unsigned char* ring = reinterpret_cast<unsigned char*>(arena);
    const uint32_t ring_lds = lds_addr(ring);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // DMA sources as byte offsets from the slab's wave-uniform base: X
    // instruction u of this wave covers tile rows (4 u + wave) 8 .. + 7, Y
    // instruction u the slab rows k = (4 u + wave) 2, + 1.
    uint32_t xoff[4], yoff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = (4 * u + wv) * 8 + (lane >> 3);
      const int c = (lane & 7) ^ ((row >> 1) & 7);
      const int64_t g = (m0 + row < M ? m0 + row : M - 1) - m0;
      xoff[u] = (uint32_t)((g * p.ldx + 4 * c) * 4);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = (4 * u + wv) * 2 + (lane >> 5);
      const int64_t col = n0 + 4 * ((lane & 31) ^ ((k & 3) << 2));
      yoff[u] = (uint32_t)(((int64_t)k * p.ldy + (col < N ? col : N - 4) - n0) * 4);
    }
    const float* xbase = X + m0 * p.ldx;
    const float* ybase = Y + n0;
    auto issue_part = [&](int kt, int h) {   // X and Y instructions 2 h, 2 h + 1
      const uint32_t st = ring_lds + (uint32_t)((kt & 1) * SB);
      const float* xb = xbase + (int64_t)kt * BK;
      const float* yb = ybase + (int64_t)kt * BK * p.ldy;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int u = 2 * h + v;
        lds_dma16s(xb, xoff[u], st + (uint32_t)((4 * u + wv) * 1024));
        lds_dma16s(yb, yoff[u], st + (uint32_t)(XB + (4 * u + wv) * 1024));
      }
    };
    // Operand byte offsets within a stage for MFMA step t (k = 4 t + lk): A
    // X[wm 64 + 16 i + lr][k] at offa[t] + 2048 i, B Y[k][wn 64 + 16 j + lr]
    // at offb[j] + 2048 t.
    const int sw = (lr >> 1) & 7;   // row permutation of every row this lane reads
    int offa[8], offb[FN];
#pragma unroll
    for (int t = 0; t < 8; ++t) offa[t] = (wm * WTM + lr) * 128 + ((t ^ sw) * 16) + 4 * lk;
#pragma unroll
    for (int j = 0; j < FN; ++j)
      offb[j] = XB + lk * 512 + ((((wn * WTN + 16 * j + lr) >> 2) ^ (lk << 2)) * 16) + 4 * (lr & 3);
    auto read_ops = [&](int kt, int t, float (&a)[FM], float (&b)[FN]) {
      const unsigned char* stage = ring + (kt & 1) * SB;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const float*>(stage + offa[t] + 2048 * i);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const float*>(stage + offb[j] + 2048 * t);
    };
    float fa[2][FM], fb[2][FN];
    if (nk > 0) {
      issue_part(0, 0);
      issue_part(0, 1);
      dma_wait_barrier<0>();
      read_ops(0, 0, fa[0], fb[0]);
    }
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
    for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (t < 7) {
          read_ops(kt, t + 1, fa[(t + 1) & 1], fb[(t + 1) & 1]);
        } else {
          // Slab kt + 1 has landed and every wave holds its slab-kt operands;
          // the reads follow on every path (after the last slab they read a
          // stage and go unused) so the compiler's LDS wait before this
          // step's MFMAs does not count them.
          dma_wait_barrier<0>();
          read_ops(kt + 1, 0, fa[0], fb[0]);
        }
        if (t < 2 && kt + 1 < nk) issue_part(kt + 1, t);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[t & 1][i], fb[t & 1][j], acc[i][j],
                                                             0, 0, 0);
        // Each step's region: the next step's LDS reads first, then its MFMAs.
        __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }
  if (nk > 0 && !DMA) load(0);
  for (int kt = 0; kt < nk && !DMA; ++kt) {
    const int buf = kt & 1;
    store(buf);
    __syncthreads();
    if (kt + 1 < nk) load((int64_t)(kt + 1) * BK);
    const float* xs = &Xs[buf][(wm * WTM + lr) * XS + lk];
    const float* ys = &Ys[buf][lk * YS + wn * WTN + lr];
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      float a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = xs[i * 16 * XS + ks];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = ys[ks * YS + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // Scheduling hint: interleave the slab's LDS reads with its MFMAs
    // (bf16 -5..9%, split -2%, float32 unchanged, measured standalone).
    __builtin_amdgcn_iglp_opt(1);
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }

  // The next fragment's addends are loaded before the current one's stores.
  double ss = 0.0;
  float e1[2][4], e2[2][4];
  auto frag_col = [&](int f) { return n0 + wn * WTN + (f % FN) * 16 + lr; };
  auto frag_rows = [&](int f) {
    const int64_t r0 = m0 + wm * WTM + (f / FN) * 16 + 4 * lk;
    return [r0](int r) { return r0 + r; };
  };
  load_addends<4>(p, frag_col(0), frag_rows(0), e1[0], e2[0]);
#pragma unroll
  for (int f = 0; f < FM * FN; ++f) {
    if (f + 1 < FM * FN)
      load_addends<4>(p, frag_col(f + 1), frag_rows(f + 1), e1[(f + 1) & 1], e2[(f + 1) & 1]);
    const int64_t col = frag_col(f);
    const auto row_of = frag_rows(f);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row_of(r);
      if (row < M && col < N)
        put(p, row, col, acc[f / FN][f % FN][r], e1[f & 1][r], e2[f & 1][r], ss);
    }
  }
  write_partial(p, ss, red, tm, tn, tiles_n);
}

// ---------------------------------------------------------------------------
// float32, NN, 256 x 256 tiles fed by LDS DMA
// ---------------------------------------------------------------------------
// Eight waves of 64 x 128 (one workgroup per CU, two waves per SIMD: one
// wave's waits hide behind the other's MFMAs).  K runs in 32-deep slabs
// that global_load_lds_dwordx4 writes into two LDS stages: a slab lands while
// the previous one is multiplied (eight k-steps of 32 MFMAs per wave), and one
// barrier per slab orders the stages.  An X row keeps K contiguous (128 B per
// row and slab), a Y row N (1 KB per k).  One 16-byte read gives a lane the A
// operands of four MFMA steps: in k-group g (16 k) lane (r, q) = (lane % 16,
// lane / 16) holds X[row][16 g + 4 q + j] for step j, so its B operand in
// step j is Y[16 g + 4 q + j][col].  One 16-byte read of a Y row gives the B
// operands of four fragments: fragment j of a wave's 64-column half takes the
// columns 4 r + j, so lane (r, q) reads columns 4 r .. 4 r + 3 of the half,
// and after the K loop it holds four adjacent columns of each output row it
// owns (stored with one 16-byte access where the output allows).  The 16-byte
// chunks of an X row are permuted, chunk c of row R at c ^ f32_xsw(R) (R mod
// 16 decides which bank half and window a lane of a 16-lane read group hits),
// so that the A reads spread over all 64 banks; the B reads do unpermuted
// (a group's lanes read 16 different chunks).  Requires K a multiple of 32,
// N a multiple of 4, row strides multiples of 4 floats and 16-byte aligned
// operands; rows past M and columns past N of edge tiles read row M - 1 and
// the last four columns instead and feed only outputs that are not stored.
constexpr int kF32DmaBK = 32;

__device__ __forceinline__ int f32_xsw(int row) { return (row & 2) | ((row >> 1) & 4); }

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
gemm_f32_nn_dma_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int BM = 256, BN = 256, BK = kF32DmaBK, NW = 8, NST = 2;
  constexpr int WTM = 64, WTN = 128, FM = WTM / 16, FN = WTN / 16;
  constexpr int XBYTES = BM * BK * 4;           // 256 rows of 128 B
  constexpr int SBYTES = XBYTES + BK * BN * 4;  // + 32 rows of 1 KB
  constexpr int XI = BM / 8 / NW;               // DMA instructions per wave and slab: X, 8 rows each
  constexpr int YI = BK / NW;                   // Y, one row each
  static_assert(XI * NW * 8 == BM && YI * NW == BK && BN == 256, "DMA split");
  __shared__ __attribute__((aligned(1024))) unsigned char ring[NST * SBYTES];
  __shared__ double red[NW];

  const float* X = static_cast<const float*>(p.X);
  const float* Y = static_cast<const float*>(p.Y);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  const uint32_t ring_lds = lds_addr(&ring[0]);

  // DMA sources, as byte offsets from the slab's wave-uniform base: X
  // instruction u of this wave covers tile rows (u NW + wave) 8 .. + 7, Y
  // instruction u slab row k = u NW + wave.
  uint32_t xoff[XI], yoff[YI];
#pragma unroll
  for (int u = 0; u < XI; ++u) {
    const int row = (u * NW + wave) * 8 + (lane >> 3);
    const int c = (lane & 7) ^ f32_xsw(row);
    const int64_t g = (m0 + row < M ? m0 + row : M - 1) - m0;
    xoff[u] = (uint32_t)((g * p.ldx + 4 * c) * 4);
  }
#pragma unroll
  for (int u = 0; u < YI; ++u) {
    const int k = u * NW + wave;
    const int64_t col = n0 + 4 * lane;
    yoff[u] = (uint32_t)(((int64_t)k * p.ldy + (col < N ? col : N - 4) - n0) * 4);
  }
  const float* xbase = X + m0 * p.ldx;
  const float* ybase = Y + n0;
  // Part h (0 .. 3) of slab kt's DMA: X instruction h and Y instruction h.
  static_assert(XI == 4 && YI == 4, "DMA parts");
  auto issue_part = [&](int kt, int h) {
    const uint32_t st = ring_lds + (uint32_t)((kt % NST) * SBYTES);
    lds_dma16s(xbase + (int64_t)kt * BK, xoff[h], st + (uint32_t)((h * NW + wave) * 1024));
    lds_dma16s(ybase + (int64_t)kt * BK * p.ldy, yoff[h],
               st + (uint32_t)(XBYTES + (h * NW + wave) * 1024));
  };

  // Operand byte offsets within a stage.  A, k-group g, fragment i (+ 2048 i):
  // row wm 64 + r, chunk 4 g + q.  B, half h of the wave's columns, step s of
  // group g (+ 256 h + 1024 (16 g + s)): row 4 q, columns wn 128 + 4 r .. + 3.
  const int r = lane & 15, q = lane >> 4;
  int offa[2];
#pragma unroll
  for (int g = 0; g < 2; ++g) offa[g] = (wm * WTM + r) * 128 + (((4 * g + q) ^ f32_xsw(r)) * 16);
  const int offb = XBYTES + q * 4096 + wn * 512 + 16 * r;

  auto read_a = [&](int kt, int g, f32x4 (&a)[FM]) {
    const unsigned char* stage = ring + (kt % NST) * SBYTES;
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *reinterpret_cast<const f32x4*>(stage + offa[g] + i * 2048);
  };
  auto read_b = [&](int kt, int t, float (&b)[FN]) {   // step t = 4 g + s of the slab
    const unsigned char* stage = ring + (kt % NST) * SBYTES + (16 * (t >> 2) + (t & 3)) * 1024;
#pragma unroll
    for (int h = 0; h < FN / 4; ++h) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(stage + offb + h * 256);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) b[4 * h + jj] = v[jj];
    }
  };

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // A is read a k-group (four steps) ahead, B a step ahead.  Slab kt + 1's
  // DMA is issued in four parts over slab kt's first four steps (all at once
  // it queues 64 instructions on the CU's address unit behind the barrier) into
  // the stage slab kt - 1 used; the barrier before slab kt's last step (every
  // wave then holds all its operands of slab kt) makes it visible and frees
  // slab kt's stage.
  const int nk = (int)(K / BK);
  f32x4 fa[2][FM];
  float fb[2][FN];
  if (nk > 0) {
#pragma unroll
    for (int h = 0; h < 4; ++h) issue_part(0, h);
    dma_wait_barrier<0>();
    read_a(0, 0, fa[0]);
    read_b(0, 0, fb[0]);
  }
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t == 0) read_a(kt, 1, fa[1]);
      if (t < 7) {
        read_b(kt, t + 1, fb[(t + 1) & 1]);
      } else {
        // Also after the last slab (the reads are then unused): with the
        // reads on every path the compiler's LDS wait before this step's
        // MFMAs does not count them.
        dma_wait_barrier<0>();
        read_a(kt + 1, 0, fa[0]);
        read_b(kt + 1, 0, fb[0]);
      }
      if (t < 4 && kt + 1 < nk) issue_part(kt + 1, t);
      const int g = t >> 2, sidx = t & 3;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[g][i][sidx], fb[t & 1][j], acc[i][j],
                                                           0, 0, 0);
      // Each step's region: the next step's LDS reads first, then its
      // MFMAs (the default schedule sinks the reads to the end of the step,
      // where their latency shows).
      __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // Output unit u = (fragment row i, column half h, element e): the lane's
  // row wm 64 + 16 i + 4 q + e and columns wn 128 + 64 h + 4 r .. + 3, the
  // values acc[i][4 h + jj][e].  Where every output and addend allows it the
  // four columns go as one 16-byte access (the bf16 copy as one 8-byte one);
  // the addends of unit u + PD are loaded before unit u's stores (loads and
  // stores complete in issue order, so a load issued after a store waits for
  // it); units by compile-time index (a run-time index would put acc in
  // scratch).
  constexpr int PD = NSR_F32_EPI_PD, NU = FM * (FN / 4) * 4;
  const bool vec = (!p.D || (((uintptr_t)p.D & 15) == 0 && (p.ldd & 3) == 0)) &&
                   (!p.Db || (((uintptr_t)p.Db & 7) == 0 && (p.lddb & 3) == 0)) &&
                   (!p.E1 || (((uintptr_t)p.E1 & 15) == 0 && (p.lde1 & 3) == 0)) &&
                   (!p.E2 || (((uintptr_t)p.E2 & 15) == 0 && (p.lde2 & 3) == 0));
  double ss = 0.0;
  f32x4 e1[PD + 1], e2[PD + 1];
  auto unit_row = [&](int u) { return m0 + wm * WTM + 16 * (u >> 3) + 4 * q + (u & 3); };
  auto unit_col = [&](int u) { return n0 + wn * WTN + 64 * ((u >> 2) & 1) + 4 * r; };
  auto load4 = [&](int u, f32x4& a1, f32x4& a2) {
    const int64_t row = unit_row(u), col = unit_col(u);
    a1 = f32x4{0.f, 0.f, 0.f, 0.f};
    a2 = a1;
    if (row >= M) return;
    if (vec && col + 3 < N) {
      if (p.E1) a1 = *reinterpret_cast<const f32x4*>(p.E1 + row * p.lde1 + col);
      if (p.E2) a2 = *reinterpret_cast<const f32x4*>(p.E2 + row * p.lde2 + col);
      return;
    }
#pragma unroll
    for (int jj = 0; jj < 4; ++jj)
      if (col + jj < N) {
        if (p.E1) a1[jj] = p.E1[row * p.lde1 + col + jj];
        if (p.E2) a2[jj] = p.E2[row * p.lde2 + col + jj];
      }
  };
  static_for<0, PD>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    load4(u, e1[u], e2[u]);
  });
  static_for<0, NU>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    if constexpr (u + PD < NU) load4(u + PD, e1[(u + PD) % (PD + 1)], e2[(u + PD) % (PD + 1)]);
    constexpr int i = u >> 3, h = (u >> 2) & 1, e = u & 3, b = u % (PD + 1);
    const int64_t row = unit_row(u), col = unit_col(u);
    if (row < M) {
      f32x4 v;
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        float x = p.scale * acc[i][4 * h + jj][e];
        if (row == col + jj) x += p.diag;
        if (p.E1) x += e1[b][jj];
        if (p.E2) x += e2[b][jj];
        v[jj] = x;
      }
      if (vec && col + 3 < N) {
        if (p.D) *reinterpret_cast<f32x4*>(p.D + row * p.ldd + col) = v;
        if (p.Db) {
          uint2 w;
          w.x = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[0]) |
                ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[1]) << 16);
          w.y = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[2]) |
                ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)v[3]) << 16);
          *reinterpret_cast<uint2*>(p.Db + row * p.lddb + col) = w;
        }
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) ss += (double)v[jj] * (double)v[jj];
      } else {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (col + jj < N) {
            if (p.D) p.D[row * p.ldd + col + jj] = v[jj];
            if (p.Db) p.Db[row * p.lddb + col + jj] = __builtin_bit_cast(uint16_t, (__bf16)v[jj]);
            ss += (double)v[jj] * (double)v[jj];
          }
      }
    }
  });
  write_partial<NW>(p, ss, red, tm, tn, tiles_n);
}

// ---------------------------------------------------------------------------
// bf16, NT: D = X Y^T, X: m x k, Y: n x k (both row-major, K contiguous)
// ---------------------------------------------------------------------------
// WGM x WGN waves per workgroup, each owning a (BM / WGM) x (BN / WGN) block.
template <int BM, int BN, int BK, bool VEC, int WGM = 2, int WGN = 2>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2)))
gemm_bf16_nt_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  constexpr int S = BK + 8;                  // LDS row stride (bf16), 16-B aligned rows
  constexpr int XV = (BM * BK / 8) / NT;     // 16-byte vectors per thread
  constexpr int YV = (BN * BK / 8) / NT;
  static_assert(XV >= 1 && YV >= 1, "tile too small");
  static_assert(XV * NT == BM * BK / 8 && YV * NT == BN * BK / 8, "slab / thread mismatch");
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][BM * S];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][BN * S];
  __shared__ double red[WGM * WGN];

  const __bf16* X = static_cast<const __bf16*>(p.X);
  const __bf16* Y = static_cast<const __bf16*>(p.Y);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  uint4 xr[XV], yr[YV];

  auto load_one = [&](const __bf16* base, int64_t ld, int64_t r0, int64_t rmax, int64_t k0,
                      int v) -> uint4 {
    {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
      const int64_t gr = r0 + row, gk = k0 + c;
      uint4 val = make_uint4(0u, 0u, 0u, 0u);
      if (gr < rmax) {
        const __bf16* src = base + gr * ld + gk;
        if (VEC && gk + 7 < K) {
          val = *reinterpret_cast<const uint4*>(src);
        } else {
          unsigned short tmp[8];
          const unsigned short* s16 = reinterpret_cast<const unsigned short*>(src);
#pragma unroll
          for (int e = 0; e < 8; ++e) tmp[e] = (gk + e < K) ? s16[e] : (unsigned short)0;
          val.x = tmp[0] | ((unsigned)tmp[1] << 16);
          val.y = tmp[2] | ((unsigned)tmp[3] << 16);
          val.z = tmp[4] | ((unsigned)tmp[5] << 16);
          val.w = tmp[6] | ((unsigned)tmp[7] << 16);
        }
      }
      return val;
    }
  };
  // Interior tiles load full slabs with unchecked 16-byte loads (wave-uniform
  // branch); edge tiles and a partial last K slab take the checked path.
  const bool interior = VEC && (m0 + BM <= M) && (n0 + BN <= N);
  auto load = [&](int64_t k0) {
    if (interior && k0 + BK <= K) {
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int idx = tid + NT * v;
        xr[v] = *reinterpret_cast<const uint4*>(X + (m0 + idx / (BK / 8)) * p.ldx + k0 +
                                                (idx % (BK / 8)) * 8);
      }
#pragma unroll
      for (int v = 0; v < YV; ++v) {
        const int idx = tid + NT * v;
        yr[v] = *reinterpret_cast<const uint4*>(Y + (n0 + idx / (BK / 8)) * p.ldy + k0 +
                                                (idx % (BK / 8)) * 8);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < XV; ++v) xr[v] = load_one(X, p.ldx, m0, M, k0, v);
#pragma unroll
    for (int v = 0; v < YV; ++v) yr[v] = load_one(Y, p.ldy, n0, N, k0, v);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
      *reinterpret_cast<uint4*>(&Xs[buf][row * S + c]) = xr[v];
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
      *reinterpret_cast<uint4*>(&Ys[buf][row * S + c]) = yr[v];
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

  const int nk = (int)((K + BK - 1) / BK);
  const int lr = lane & 31, lk = lane >> 5;
  if (nk > 0) load(0);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    store(buf);
    __syncthreads();
    if (kt + 1 < nk) load((int64_t)(kt + 1) * BK);
    const __bf16* xs = &Xs[buf][(wm * WTM + lr) * S + 8 * lk];
    const __bf16* ys = &Ys[buf][(wn * WTN + lr) * S + 8 * lk];
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8*>(xs + i * 32 * S + ks);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const bf16x8*>(ys + j * 32 * S + ks);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // Scheduling hint: interleave the slab's LDS reads with its MFMAs
    // (bf16 -5..9%, split -2%, float32 unchanged, measured standalone).
    __builtin_amdgcn_iglp_opt(1);
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }

  // Half a fragment's addends (2 x 8) are loaded together before its stores
  // (the 256-register budget of two waves per SIMD leaves no room for more):
  // one memory round trip per half fragment.  Without addends the stores
  // run back to back.
  double ss = 0.0;
  if (!p.E1 && !p.E2) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int64_t col = n0 + wn * WTN + j * 32 + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
          if (row < M && col < N) put(p, row, col, acc[i][j][r], 0.0f, 0.0f, ss);
        }
      }
  } else {
#pragma unroll
    for (int f = 0; f < FM * FN; ++f) {
      const int64_t col = n0 + wn * WTN + (f % FN) * 32 + lr;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t r0 = m0 + wm * WTM + (f / FN) * 32 + 16 * h + 4 * lk;
        const auto row_of = [r0](int r) { return r0 + 8 * (r >> 2) + (r & 3); };
        float e1[8], e2[8];
        load_addends<8>(p, col, row_of, e1, e2);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int64_t row = row_of(r);
          if (row < M && col < N)
            put(p, row, col, acc[f / FN][f % FN][8 * h + r], e1[r], e2[r], ss);
        }
      }
    }
  }
  write_partial<WGM * WGN>(p, ss, red, tm, tn, tiles_n);
}

// ---------------------------------------------------------------------------
// bf16, NT, 256 x 256 tiles fed by LDS DMA (global_load_lds_dwordx4): the
// K slabs (64 deep in two LDS stages, or 32 deep in four) go from global
// memory straight into a ring of LDS stages, ahead of the MFMAs, with no
// register staging and no LDS store phase between slabs; one barrier per
// slab.  Eight waves of 128 x 64 as in gemm_bf16_nt_kernel<256, 256>, same
// epilogue.
//
// LDS layout of a stage: X rows then Y rows, BK bf16 per row, the row's
// 16-byte chunks permuted by chunk ^ swz(row).  A 128-bit LDS read is
// serviced sixteen lanes (256 bytes, all 64 banks) at a time, in the groups
// {0-3, 12-15, 20-23, 24-27} and {4-7, 8-11, 16-19, 28-31} (and the same
// + 32), as measured with bank-conflict counters on two-lane probes.  In an
// MFMA operand read, lane l reads row l % 32, one chunk for all; the
// swizzle puts a group's sixteen 16-byte reads in sixteen different bank
// quads (padded 144-byte rows have the same property).  A DMA instruction
// writes 64 x 16 bytes at m0 + 16 * lane; lane p of an instruction covering
// rows r0 .. fetches chunk (p % CH) ^ swz(row) of row r0 + p / CH, which
// lands in slot p % CH of that row.
//
// Requirements (checked by the launcher): K a multiple of 32, leading
// dimensions multiples of 8 elements and 16-byte aligned operands.  Rows
// past M (or N) of edge tiles read row M - 1 (N - 1) instead: they only feed
// outputs that are not stored.
// ---------------------------------------------------------------------------
constexpr int kDmaBK = 32;          // K per stage of the default instantiation

// Chunk permutation of a row of CH 16-byte chunks (CH = 4: 32 bf16 of K,
// rows of 64 bytes; CH = 8: 64 bf16, rows of 128 bytes).  The rows of a
// 16-lane read group that share a 256-byte bank window position (equal
// row % 4, resp. row % 2) differ in bits 3 and 4 (resp. 1, 3 and 4), which
// the permutation maps to different chunks (see above).
template <int CH>
__device__ __forceinline__ int dma_swz(int row) {
  return CH == 4 ? (row >> 3) & 3 : ((row >> 1) & 1) | ((row >> 2) & 6);
}

// BM x BN tile, waves of (BM / 2) x 64, NST stages of BK-deep slabs in LDS.
// BM = 256: BN = 256 is eight waves, one workgroup per CU; BN = 128 four
// waves, two workgroups per CU.  BM = BN = 128: four waves of 64 x 64, two
// workgroups per CU (64 KB of LDS each), for outputs too small to fill the
// CUs with 256-row tiles.  The library launches <256, 2, 64> when K is a
// multiple of 64 (half the barriers of <256, 4, 32>, one slab of prefetch:
// 2-4% faster at N = 4096 and 8192), else <256, 4, 32> (the same pair with
// BM = 128 for 128 x 128 tiles).  <128, 3, 32> with 256 rows (two workgroups
// per CU, 72 KB each) measured 15% slower than <256, 2, 64>.
template <int BN, int NST, int BK, int BM = 256>
__global__ void __launch_bounds__(64 * 2 * (BN / 64)) __attribute__((amdgpu_waves_per_eu(2)))
gemm_bf16_nt_dma_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int WGN = BN / 64, NW = 2 * WGN;
  constexpr int WTM = BM / 2, WTN = 64, FM = WTM / 32, FN = 2;
  constexpr int RB = BK * 2;                 // row bytes
  constexpr int CH = BK / 8;                 // 16-byte chunks per row
  constexpr int RPI = 64 / CH;               // rows per DMA instruction
  constexpr int T = BK / 16;                 // MFMA k-steps per slab
  constexpr int XBYTES = BM * RB;
  constexpr int SBYTES = XBYTES + BN * RB;
  constexpr int XI = (BM / RPI) / NW, YI = (BN / RPI) / NW;   // DMA instructions per wave and slab
  constexpr int PER = XI + YI;
  static_assert(XI * NW * RPI == BM && YI * NW * RPI == BN, "DMA split");
  static_assert(T % 2 == 0, "operand buffers alternate by step parity");
  __shared__ __attribute__((aligned(1024))) unsigned char ring[NST * SBYTES];
  __shared__ double red[NW];

  const __bf16* X = static_cast<const __bf16*>(p.X);
  const __bf16* Y = static_cast<const __bf16*>(p.Y);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  const uint32_t ring_lds = lds_addr(&ring[0]);

  // DMA sources: instruction u of this wave covers rows (u NW + wave) * RPI
  // .. + RPI - 1 of the X (u < XI) or the Y block.
  const __bf16* xsrc[XI];
  const __bf16* ysrc[YI];
#pragma unroll
  for (int u = 0; u < XI; ++u) {
    const int row = (u * NW + wave) * RPI + lane / CH;
    const int c = (lane % CH) ^ dma_swz<CH>(row);
    const int64_t g = m0 + row < M ? m0 + row : M - 1;
    xsrc[u] = X + g * p.ldx + 8 * c;
  }
#pragma unroll
  for (int u = 0; u < YI; ++u) {
    const int row = (u * NW + wave) * RPI + lane / CH;
    const int c = (lane % CH) ^ dma_swz<CH>(row);
    const int64_t g = n0 + row < N ? n0 + row : N - 1;
    ysrc[u] = Y + g * p.ldy + 8 * c;
  }
  auto issue = [&](int kt) {
    const uint32_t st = ring_lds + (uint32_t)((kt % NST) * SBYTES);
    const int64_t k0 = (int64_t)kt * BK;
#pragma unroll
    for (int u = 0; u < XI; ++u)
      lds_dma16(xsrc[u] + k0, st + (uint32_t)((u * NW + wave) * 1024));
#pragma unroll
    for (int u = 0; u < YI; ++u)
      lds_dma16(ysrc[u] + k0, st + (uint32_t)(XBYTES + (u * NW + wave) * 1024));
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

  const int lr = lane & 31, lk = lane >> 5;
  const int sw = dma_swz<CH>(lr);   // = dma_swz of every row this lane reads
  // Byte offsets (within a stage) of this lane's operand chunks for the T
  // 16-deep MFMA steps of a slab; fragment i / j adds 32 rows.
  int offa[T], offb[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int chunk = ((2 * t + lk) ^ sw) * 16;
    offa[t] = (wm * WTM + lr) * RB + chunk;
    offb[t] = XBYTES + (wn * WTN + lr) * RB + chunk;
  }

  const int nk = (int)(K / BK);
  // Slab s has landed everywhere once at most the DMAs of the slabs issued
  // after it (up to NST - 2 of them, PER instructions each) are outstanding;
  // the lgkmcnt(0) before the barrier makes this wave's operand reads of the
  // stage that the next DMA overwrites complete first.
  auto wait_slab = [&](int s) {
    const int later = min(NST - 2, nk - 1 - s);
    if (later >= 2)
      dma_wait_barrier<2 * PER>();
    else if (later == 1)
      dma_wait_barrier<PER>();
    else
      dma_wait_barrier<0>();
  };
  auto read_frags = [&](int s, int t, bf16x8 (&a)[FM], bf16x8 (&b)[FN]) {
    const unsigned char* stage = ring + (s % NST) * SBYTES;
#pragma unroll
    for (int i = 0; i < FM; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(stage + offa[t] + i * 32 * RB);
#pragma unroll
    for (int j = 0; j < FN; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(stage + offb[t] + j * 32 * RB);
  };
  auto mfmas = [&](const bf16x8 (&a)[FM], const bf16x8 (&b)[FN]) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  };
  // Pipeline: the DMA of slab s + NST - 1 is issued right after the barrier
  // that confirms slab s; each step's operands are read before the previous
  // step's MFMAs (across the slab boundary too), so their LDS latency hides
  // behind them.
  if (nk > 0) {
#pragma unroll
    for (int s = 0; s < NST - 1; ++s)
      if (s < nk) issue(s);
    wait_slab(0);
    if (NST - 1 < nk) issue(NST - 1);
  }
  bf16x8 fa[2][FM], fb[2][FN];
  if (nk > 0) read_frags(0, 0, fa[0], fb[0]);
  if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (t + 1 < T) {
        read_frags(kt, t + 1, fa[(t + 1) & 1], fb[(t + 1) & 1]);
      } else {
        // Also after the last slab (the reads are then unused): with the
        // reads on every path the compiler's LDS wait before this step's
        // MFMAs does not count them.
        wait_slab(kt + 1);
        if (kt + NST < nk) issue(kt + NST);
        read_frags(kt + 1, 0, fa[0], fb[0]);
      }
      mfmas(fa[t & 1], fb[t & 1]);
      // Each step's region: the next step's LDS reads first, then its MFMAs.
      __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);

  double ss = 0.0;
  if (!p.E1 && !p.E2) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int64_t col = n0 + wn * WTN + j * 32 + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
          if (row < M && col < N) put(p, row, col, acc[i][j][r], 0.0f, 0.0f, ss);
        }
      }
  } else {
    // Chunks of four rows of one fragment column; the addends of chunk c + PD
    // are loaded before chunk c's stores (loads and stores complete in issue
    // order, so a load issued after a store waits for it), and the chunks go
    // by compile-time index (a run-time one puts acc in scratch).
    constexpr int NC = FM * FN * 4, PD = NSR_BF16_EPI_PD;
    auto chunk_col = [&](int c) { return n0 + wn * WTN + ((c >> 2) % FN) * 32 + lr; };
    auto chunk_r0 = [&](int c) {
      return m0 + wm * WTM + ((c >> 2) / FN) * 32 + 8 * (c & 3) + 4 * lk;
    };
    float e1[PD + 1][4], e2[PD + 1][4];
    static_for<0, PD>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      const int64_t q0 = chunk_r0(c);
      load_addends<4>(p, chunk_col(c), [q0](int r) { return q0 + r; }, e1[c], e2[c]);
    });
    static_for<0, NC>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if constexpr (c + PD < NC) {
        const int64_t qn = chunk_r0(c + PD);
        load_addends<4>(p, chunk_col(c + PD), [qn](int r) { return qn + r; },
                        e1[(c + PD) % (PD + 1)], e2[(c + PD) % (PD + 1)]);
      }
      const int64_t col = chunk_col(c), q = chunk_r0(c);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = q + r;
        if (row < M && col < N)
          put(p, row, col, acc[(c >> 2) / FN][(c >> 2) % FN][4 * (c & 3) + r],
              e1[c % (PD + 1)][r], e2[c % (PD + 1)][r], ss);
      }
    });
  }
  write_partial<NW>(p, ss, red, tm, tn, tiles_n);
}

// ---------------------------------------------------------------------------
// float32-class product from split half-precision operands
// ---------------------------------------------------------------------------
// A float32 operand scaled by 2^e (max |x| 2^e in [2^14, 2^15), inside the
// half-precision range) is written as hi + lo with hi = half(x 2^e) and
// lo = half(x 2^e - hi); x 2^e - hi is exact in float32 and below 2^-11 of
// |x 2^e|, so hi + lo keeps 22 significant bits.  X Y^T then takes three
// half-precision products, hi hi^T + hi lo^T + lo hi^T (the dropped lo lo^T
// is below 2^-22 relative), accumulated in float32.

// Exponent of the split scale from per-block maxima (every thread of the
// block returns the same value): 0 for a zero or non-finite maximum, so
// infinities and NaNs reach the output unchanged.
__device__ int split_exponent(const float* part, int64_t nparts, float* red) {
  float m = 0.0f;
  for (int64_t i = threadIdx.x; i < nparts; i += blockDim.x) m = fmaxf(m, part[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  float t = 0.0f;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmaxf(t, red[w]);
  if (!(t > 0.0f) || !(t < INFINITY)) return 0;
  const int e = 14 - ilogbf(t);
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

__device__ __forceinline__ void split_one(float x, float s, uint16_t& h, uint16_t& l) {
  const float xs = x * s;
  const _Float16 hh = (_Float16)xs;
  const _Float16 ll = (_Float16)(xs - (float)hh);
  h = __builtin_bit_cast(uint16_t, hh);
  l = __builtin_bit_cast(uint16_t, ll);
}

__global__ void __launch_bounds__(256) absmax_kernel(const float* X, int64_t ld, int64_t rows,
                                                     int64_t cols, bool vec, float* part) {
  __shared__ float red[4];
  float m = 0.0f;
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const float* row = X + r * ld;
    if (vec) {
      const int64_t c4 = cols >> 2;
      for (int64_t c = threadIdx.x; c < c4; c += 256) {
        const float4 v = reinterpret_cast<const float4*>(row)[c];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
      }
      for (int64_t c = (c4 << 2) + threadIdx.x; c < cols; c += 256) m = fmaxf(m, fabsf(row[c]));
    } else {
      for (int64_t c = threadIdx.x; c < cols; c += 256) m = fmaxf(m, fabsf(row[c]));
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

// Row-major planes: each thread splits 8 consecutive elements of a row.
__global__ void __launch_bounds__(256) split_rows_kernel(const float* X, int64_t ld, int64_t rows,
                                                         int64_t cols, bool vec, const float* part,
                                                         int64_t nparts, uint16_t* hi,
                                                         uint16_t* lo, int64_t ldh,
                                                         float* exp_out) {
  __shared__ float red[4];
  const int e = split_exponent(part, nparts, red);
  const float s = ldexpf(1.0f, e);
  if (blockIdx.x == 0 && threadIdx.x == 0) exp_out[0] = (float)e;
  const int64_t c8 = (cols + 7) >> 3;
  const int64_t total = rows * c8;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * 256) {
    const int64_t r = q / c8, c = (q - r * c8) * 8;
    const float* src = X + r * ld + c;
    const bool full = c + 8 <= cols;
    float v[8];
    if (vec && full) {
      const float4 a = reinterpret_cast<const float4*>(src)[0];
      const float4 b = reinterpret_cast<const float4*>(src)[1];
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i) v[i] = (c + i < cols) ? src[i] : 0.0f;
    }
    uint16_t h[8], l[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) split_one(v[i], s, h[i], l[i]);
    uint16_t* dh = hi + r * ldh + c;
    uint16_t* dl = lo + r * ldh + c;
    if (full) {
      uint4 ph, pl;
      ph.x = h[0] | ((unsigned)h[1] << 16); ph.y = h[2] | ((unsigned)h[3] << 16);
      ph.z = h[4] | ((unsigned)h[5] << 16); ph.w = h[6] | ((unsigned)h[7] << 16);
      pl.x = l[0] | ((unsigned)l[1] << 16); pl.y = l[2] | ((unsigned)l[3] << 16);
      pl.z = l[4] | ((unsigned)l[5] << 16); pl.w = l[6] | ((unsigned)l[7] << 16);
      *reinterpret_cast<uint4*>(dh) = ph;
      *reinterpret_cast<uint4*>(dl) = pl;
    } else {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (c + i < cols) {
          dh[i] = h[i];
          dl[i] = l[i];
        }
    }
  }
}

// Transposed planes: a 64 x 64 tile of X goes through LDS; output row j of
// the planes is column j of X.
__global__ void __launch_bounds__(256) split_trans_kernel(const float* X, int64_t ld,
                                                          int64_t rows, int64_t cols, bool vec,
                                                          const float* part, int64_t nparts,
                                                          uint16_t* hi, uint16_t* lo,
                                                          int64_t ldh, float* exp_out) {
  __shared__ float red[4];
  __shared__ float tile[64][65];
  const int e = split_exponent(part, nparts, red);
  const float s = ldexpf(1.0f, e);
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) exp_out[0] = (float)e;
  const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = tid + 256 * i;
    const int row = idx >> 4, c4 = (idx & 15) * 4;
    const int64_t gr = r0 + row, gc = c0 + c4;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (gr < rows) {
      const float* src = X + gr * ld + gc;
      if (vec && gc + 4 <= cols) {
        v = *reinterpret_cast<const float4*>(src);
      } else {
        if (gc < cols) v.x = src[0];
        if (gc + 1 < cols) v.y = src[1];
        if (gc + 2 < cols) v.z = src[2];
        if (gc + 3 < cols) v.w = src[3];
      }
    }
    tile[row][c4] = v.x;
    tile[row][c4 + 1] = v.y;
    tile[row][c4 + 2] = v.z;
    tile[row][c4 + 3] = v.w;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int q = tid + 256 * i;
    const int j = q >> 3, k8 = (q & 7) * 8;
    const int64_t orow = c0 + j, ocol = r0 + k8;
    if (orow >= cols) continue;
    uint16_t h[8], l[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) split_one(tile[k8 + t][j], s, h[t], l[t]);
    uint16_t* dh = hi + orow * ldh + ocol;
    uint16_t* dl = lo + orow * ldh + ocol;
    if (ocol + 8 <= rows) {
      uint4 ph, pl;
      ph.x = h[0] | ((unsigned)h[1] << 16); ph.y = h[2] | ((unsigned)h[3] << 16);
      ph.z = h[4] | ((unsigned)h[5] << 16); ph.w = h[6] | ((unsigned)h[7] << 16);
      pl.x = l[0] | ((unsigned)l[1] << 16); pl.y = l[2] | ((unsigned)l[3] << 16);
      pl.z = l[4] | ((unsigned)l[5] << 16); pl.w = l[6] | ((unsigned)l[7] << 16);
      *reinterpret_cast<uint4*>(dh) = ph;
      *reinterpret_cast<uint4*>(dl) = pl;
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (ocol + t < rows) {
          dh[t] = h[t];
          dl[t] = l[t];
        }
    }
  }
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// Physical 16-byte chunk of logical chunk c in LDS row `row` (rows of BK
// halves, no padding): XORed with bits of the row so that eight consecutive
// lanes hit eight different bank groups both when a slab is stored (BK / 8
// chunks of a row per lane group) and when a fragment is read (one chunk of
// eight consecutive rows).
template <int BK>
__device__ __forceinline__ int swz_chunk(int row, int c) {
  constexpr int CPR = BK / 8;                         // chunks per row
  constexpr int SH = CPR == 2 ? 2 : (CPR == 4 ? 1 : 0);
  return c ^ ((row >> SH) & (CPR - 1));
}

// D = X Y^T from split planes; tiling as in the bf16 NT kernel, with the
// high and low planes of each operand staged side by side in LDS.
template <int BM, int BN, int BK, bool VEC, int WGM = 2, int WGN = 2>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2)))
gemm_f16s_nt_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int NT = 64 * WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  static_assert(BK == 16 || BK == 32 || BK == 64, "swizzle defined for 2, 4, 8 chunks per row");
  constexpr int S = BK;                      // LDS row stride (halves), chunks swizzled
  constexpr int XV = (BM * BK / 8) / NT;     // 16-byte vectors per thread and plane
  constexpr int YV = (BN * BK / 8) / NT;
  static_assert(XV >= 1 && YV >= 1, "tile too small");
  static_assert(XV * NT == BM * BK / 8 && YV * NT == BN * BK / 8, "slab / thread mismatch");
  __shared__ __attribute__((aligned(16))) _Float16 Xs[2][2][BM * S];  // [buffer][hi, lo]
  __shared__ __attribute__((aligned(16))) _Float16 Ys[2][2][BN * S];
  __shared__ double red[WGM * WGN];

  const uint16_t* Xp[2] = {static_cast<const uint16_t*>(p.X), static_cast<const uint16_t*>(p.Xl)};
  const uint16_t* Yp[2] = {static_cast<const uint16_t*>(p.Y), static_cast<const uint16_t*>(p.Yl)};
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;
  uint4 xr[2][XV], yr[2][YV];

  auto load_one = [&](const uint16_t* base, int64_t ld, int64_t r0, int64_t rmax, int64_t k0,
                      int v) -> uint4 {
    const int idx = tid + NT * v;
    const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
    const int64_t gr = r0 + row, gk = k0 + c;
    uint4 val = make_uint4(0u, 0u, 0u, 0u);
    if (gr < rmax) {
      const uint16_t* src = base + gr * ld + gk;
      if (VEC && gk + 7 < K) {
        val = *reinterpret_cast<const uint4*>(src);
      } else {
        unsigned short tmp[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) tmp[e] = (gk + e < K) ? src[e] : (unsigned short)0;
        val.x = tmp[0] | ((unsigned)tmp[1] << 16);
        val.y = tmp[2] | ((unsigned)tmp[3] << 16);
        val.z = tmp[4] | ((unsigned)tmp[5] << 16);
        val.w = tmp[6] | ((unsigned)tmp[7] << 16);
      }
    }
    return val;
  };
  const bool interior = VEC && (m0 + BM <= M) && (n0 + BN <= N);
  auto load = [&](int64_t k0) {
    if (interior && k0 + BK <= K) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int v = 0; v < XV; ++v) {
          const int idx = tid + NT * v;
          xr[h][v] = *reinterpret_cast<const uint4*>(Xp[h] + (m0 + idx / (BK / 8)) * p.ldx +
                                                     k0 + (idx % (BK / 8)) * 8);
        }
#pragma unroll
        for (int v = 0; v < YV; ++v) {
          const int idx = tid + NT * v;
          yr[h][v] = *reinterpret_cast<const uint4*>(Yp[h] + (n0 + idx / (BK / 8)) * p.ldy +
                                                     k0 + (idx % (BK / 8)) * 8);
        }
      }
      return;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int v = 0; v < XV; ++v) xr[h][v] = load_one(Xp[h], p.ldx, m0, M, k0, v);
#pragma unroll
      for (int v = 0; v < YV; ++v) yr[h][v] = load_one(Yp[h], p.ldy, n0, N, k0, v);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int idx = tid + NT * v;
        const int row = idx / (BK / 8), c = swz_chunk<BK>(row, idx % (BK / 8)) * 8;
        *reinterpret_cast<uint4*>(&Xs[buf][h][row * S + c]) = xr[h][v];
      }
#pragma unroll
      for (int v = 0; v < YV; ++v) {
        const int idx = tid + NT * v;
        const int row = idx / (BK / 8), c = swz_chunk<BK>(row, idx % (BK / 8)) * 8;
        *reinterpret_cast<uint4*>(&Ys[buf][h][row * S + c]) = yr[h][v];
      }
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

  const int nk = (int)((K + BK - 1) / BK);
  const int lr = lane & 31, lk = lane >> 5;
  if (nk > 0) load(0);
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    store(buf);
    __syncthreads();
    if (kt + 1 < nk) load((int64_t)(kt + 1) * BK);
    // Fragment rows are lr + multiples of 32, so the swizzle depends on lr
    // only.
    const int xo = (wm * WTM + lr) * S;
    const int yo = (wn * WTN + lr) * S;
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int co = swz_chunk<BK>(lr, ks / 8 + lk) * 8;
      f16x8 ah[FM], al[FM], bh[FN], bl[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ah[i] = *reinterpret_cast<const f16x8*>(&Xs[buf][0][xo + i * 32 * S + co]);
        al[i] = *reinterpret_cast<const f16x8*>(&Xs[buf][1][xo + i * 32 * S + co]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        bh[j] = *reinterpret_cast<const f16x8*>(&Ys[buf][0][yo + j * 32 * S + co]);
        bl[j] = *reinterpret_cast<const f16x8*>(&Ys[buf][1][yo + j * 32 * S + co]);
      }
      // Small terms first; each accumulator gets FM x FN independent
      // products between its updates.
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al[i], bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[i], bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
    // Scheduling hint: interleave the slab's LDS reads with its MFMAs
    // (bf16 -5..9%, split -2%, float32 unchanged, measured standalone).
    __builtin_amdgcn_iglp_opt(1);
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }

  // Undo the operand scales (powers of two: exact unless the result
  // underflows), then the shared epilogue.
  const float fx = p.xexp ? ldexpf(1.0f, -(int)p.xexp[0]) : 1.0f;
  const float fy = p.yexp ? ldexpf(1.0f, -(int)p.yexp[0]) : 1.0f;
  double ss = 0.0;
  if (!p.E1 && !p.E2) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int64_t col = n0 + wn * WTN + j * 32 + lr;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * WTM + i * 32 + 8 * (r >> 2) + 4 * lk + (r & 3);
          if (row < M && col < N) put(p, row, col, acc[i][j][r] * fx * fy, 0.0f, 0.0f, ss);
        }
      }
  } else {
#pragma unroll
    for (int f = 0; f < FM * FN; ++f) {
      const int64_t col = n0 + wn * WTN + (f % FN) * 32 + lr;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t r0 = m0 + wm * WTM + (f / FN) * 32 + 16 * h + 4 * lk;
        const auto row_of = [r0](int r) { return r0 + 8 * (r >> 2) + (r & 3); };
        float e1[8], e2[8];
        load_addends<8>(p, col, row_of, e1, e2);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int64_t row = row_of(r);
          if (row < M && col < N)
            put(p, row, col, acc[f / FN][f % FN][8 * h + r] * fx * fy, e1[r], e2[r], ss);
        }
      }
    }
  }
  write_partial<WGM * WGN>(p, ss, red, tm, tn, tiles_n);
}

// Split half-precision NT product, BM x BM tiles fed by LDS DMA: the bf16
// DMA kernel's layout with four operand planes (X hi, X lo, Y hi, Y lo; rows
// of 64 bytes, 32 K per slab, chunks permuted by dma_swz<4>) and three MFMA
// products per 16-k step.  BM = 256: eight waves of 128 x 64, two 64 KB
// stages, one workgroup per CU; BM = 128: four waves of 64 x 64, two 32 KB
// stages, two workgroups per CU.  The DMA sources are a wave-uniform plane
// base plus 32-bit per-lane offsets.  Requires K a multiple of 32, row
// strides multiples of 8 halves and 16-byte aligned planes.
constexpr int kF16sDmaBK = 32;

template <int BM>
__global__ void __launch_bounds__(BM == 256 ? 512 : 256) __attribute__((amdgpu_waves_per_eu(2)))
gemm_f16s_nt_dma_kernel(GemmLpArgs p, int tiles_m, int tiles_n) {
  constexpr int BK = kF16sDmaBK, NST = 2, NW = BM == 256 ? 8 : 4, WGN = BM / 64;
  constexpr int WTM = BM / 2, WTN = 64, FM = WTM / 32, FN = 2;
  constexpr int RB = BK * 2, CH = BK / 8, RPI = 64 / CH, T = BK / 16;
  constexpr int PB = BM * RB;                   // bytes of one plane's slab
  constexpr int SBYTES = 4 * PB;                // X hi, X lo, Y hi, Y lo
  constexpr int PI = (BM / RPI) / NW;           // DMA instructions per wave, plane and slab
  static_assert(NW == 2 * WGN && PI * NW * RPI == BM && T == 2, "DMA split");
  __shared__ __attribute__((aligned(1024))) unsigned char ring[NST * SBYTES];
  __shared__ double red[NW];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WGN, wn = wave % WGN;
  int tm, tn;
  map_tile_lp(blockIdx.x, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BM;
  const int64_t M = p.M, N = p.N, K = p.K;
  const uint32_t ring_lds = lds_addr(&ring[0]);

  // Plane bases at the tile's first row (wave-uniform) and per-lane byte
  // offsets: instruction u of this wave covers tile rows (u NW + wave) RPI
  // .. + RPI - 1 of each plane.
  const uint16_t* base[4] = {
      static_cast<const uint16_t*>(p.X) + m0 * p.ldx, static_cast<const uint16_t*>(p.Xl) + m0 * p.ldx,
      static_cast<const uint16_t*>(p.Y) + n0 * p.ldy, static_cast<const uint16_t*>(p.Yl) + n0 * p.ldy};
  uint32_t xoff[PI], yoff[PI];
#pragma unroll
  for (int u = 0; u < PI; ++u) {
    const int row = (u * NW + wave) * RPI + lane / CH;
    const int c = (lane % CH) ^ dma_swz<CH>(row);
    const int64_t gx = (m0 + row < M ? m0 + row : M - 1) - m0;
    const int64_t gy = (n0 + row < N ? n0 + row : N - 1) - n0;
    xoff[u] = (uint32_t)((gx * p.ldx + 8 * c) * 2);
    yoff[u] = (uint32_t)((gy * p.ldy + 8 * c) * 2);
  }
  auto issue = [&](int kt) {
    const uint32_t st = ring_lds + (uint32_t)((kt % NST) * SBYTES);
    const int64_t k0 = (int64_t)kt * BK;
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int u = 0; u < PI; ++u)
        lds_dma16s(base[h] + k0, h < 2 ? xoff[u] : yoff[u],
                   st + (uint32_t)(h * PB + (u * NW + wave) * 1024));
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

  const int lr = lane & 31, lk = lane >> 5;
  const int sw = dma_swz<CH>(lr);
  int offa[T], offb[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int chunk = ((2 * t + lk) ^ sw) * 16;
    offa[t] = (wm * WTM + lr) * RB + chunk;
    offb[t] = 2 * PB + (wn * WTN + lr) * RB + chunk;
  }
  struct Ops {
    f16x8 ah[FM], al[FM], bh[FN], bl[FN];
  };
  auto read_ops = [&](int s, int t, Ops& o) {
    const unsigned char* stage = ring + (s % NST) * SBYTES;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      o.ah[i] = *reinterpret_cast<const f16x8*>(stage + offa[t] + i * 32 * RB);
      o.al[i] = *reinterpret_cast<const f16x8*>(stage + PB + offa[t] + i * 32 * RB);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      o.bh[j] = *reinterpret_cast<const f16x8*>(stage + offb[t] + j * 32 * RB);
      o.bl[j] = *reinterpret_cast<const f16x8*>(stage + PB + offb[t] + j * 32 * RB);
    }
  };
  auto mfmas = [&](const Ops& o) {
    // Small terms first; each accumulator gets FM x FN independent products
    // between its updates.
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.al[i], o.bh[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.ah[i], o.bl[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(o.ah[i], o.bh[j], acc[i][j], 0, 0, 0);
  };

  // Slab kt + 1's DMA is issued right after the barrier that confirms slab
  // kt (every wave then holds its operands of slab kt - 1, whose stage it
  // overwrites); each step's operands are read before the previous step's
  // MFMAs, across the slab boundary too, and the boundary reads are issued
  // on every path (see the bf16 kernel).
  const int nk = (int)(K / BK);
  Ops o[2];
  if (nk > 0) {
    issue(0);
    dma_wait_barrier<0>();
    if (nk > 1) issue(1);
    read_ops(0, 0, o[0]);
  }
  if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      if (t + 1 < T) {
        read_ops(kt, t + 1, o[(t + 1) & 1]);
      } else {
        dma_wait_barrier<0>();
        if (kt + 2 < nk) issue(kt + 2);
        read_ops(kt + 1, 0, o[0]);
      }
      mfmas(o[t & 1]);
      __builtin_amdgcn_sched_group_barrier(0x100, 2 * (FM + FN), 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * FM * FN, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);

  // Undo the operand scales (powers of two: exact unless the result
  // underflows), then the shared epilogue.
  const float fx = p.xexp ? ldexpf(1.0f, -(int)p.xexp[0]) : 1.0f;
  const float fy = p.yexp ? ldexpf(1.0f, -(int)p.yexp[0]) : 1.0f;
  double ss = 0.0;
#pragma unroll
  for (int f = 0; f < FM * FN; ++f) {
    const int64_t col = n0 + wn * WTN + (f % FN) * 32 + lr;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r0 = m0 + wm * WTM + (f / FN) * 32 + 16 * h + 4 * lk;
      const auto row_of = [r0](int r) { return r0 + 8 * (r >> 2) + (r & 3); };
      float e1[8], e2[8];
      load_addends<8>(p, col, row_of, e1, e2);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t row = row_of(r);
        if (row < M && col < N)
          put(p, row, col, acc[f / FN][f % FN][8 * h + r] * fx * fy, e1[r], e2[r], ss);
      }
    }
  }
  write_partial<NW>(p, ss, red, tm, tn, tiles_n);
}

// ---------------------------------------------------------------------------
// bf16, NT, symmetric output
// ---------------------------------------------------------------------------
// The solver's bf16 products are polynomials in F, symmetric in exact
// arithmetic, so only the T (T + 1) / 2 tiles on or above the diagonal are
// computed and the lower triangle is their mirror, as in the float64 GEMM.
// Grid: the first dp workgroups own whole tiles; when the tiles leave a
// partial last round of resident workgroups, each of its tiles is cut into
// `splits` K-slices run by the remaining workgroups, which store raw
// accumulators; gemm_bf16_sym_fixup adds the slices in slice order
// (deterministic) and finishes those tiles.
constexpr int kStage = 32 * 33;            // per-wave mirror stage (floats)

__device__ __forceinline__ void sym_tile_lp(int t, int T, int& tm, int& tn) {
  int r = t, m = 0;
  while (r >= T - m) {
    r -= T - m;
    ++m;
  }
  tm = m;
  tn = m + r;
}

// Finish tile (tm <= tn) from its accumulators: elements on or above the
// diagonal get the fused terms and are stored (D, Db); an off-diagonal tile
// also writes its transpose, fragment by fragment through a per-wave LDS
// stage (32 x 33 floats) so that the mirrored rows are stored contiguously;
// a diagonal tile mirrors its strict upper triangle element by element.
// Returns this thread's sum of squares of everything it stored.  Contains
// barriers: every thread of the workgroup calls it.
template <int BM, int WGM, int WGN>
__device__ double sym_epilogue(const GemmLpArgs& p, int tm, int tn,
                               f32x16 (&acc)[BM / WGM / 32][BM / WGN / 32], float* stage) {
  constexpr int WTM = BM / WGM, WTN = BM / WGN, FM = WTM / 32, FN = WTN / 32;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lr = lane & 31, lk = lane >> 5;
  const int64_t M = p.M, N = p.N;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BM;
  const bool diag_tile = tm == tn;
  double ss = 0.0;
#pragma unroll
  for (int f = 0; f < FM * FN; ++f) {
    const int i = f / FN, j = f % FN;
    const int64_t R0 = m0 + wm * WTM + i * 32, C0 = n0 + wn * WTN + j * 32;
    const int64_t col = C0 + lr;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t r0 = R0 + 16 * h + 4 * lk;
      const auto row_of = [r0](int r) { return r0 + 8 * (r >> 2) + (r & 3); };
      float e1[8], e2[8];
      load_addends<8>(p, col, row_of, e1, e2);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int64_t row = row_of(r);
        if (row >= M || col >= N || (diag_tile && row > col)) continue;
        float v = p.scale * acc[i][j][8 * h + r];
        if (row == col) v += p.diag;
        if (p.E1) v += e1[r];
        if (p.E2) v += e2[r];
        if (p.D) p.D[row * p.ldd + col] = v;
        if (p.Db) p.Db[row * p.lddb + col] = __builtin_bit_cast(uint16_t, (__bf16)v);
        ss += (double)v * (double)v;
        if (!diag_tile) {
          stage[lr * 33 + (int)(row - R0)] = v;
        } else if (row < col) {
          if (p.D) p.D[col * p.ldd + row] = v;
          if (p.Db) p.Db[col * p.lddb + row] = __builtin_bit_cast(uint16_t, (__bf16)v);
          ss += (double)v * (double)v;
        }
      }
    }
    if (!diag_tile) {
      __syncthreads();
      // mirrored rows, two per pass (lanes 0-31 and 32-63)
      for (int c = 0; c < 32; c += 2) {
        const int ci = c + lk;
        const int64_t grow = C0 + ci, gcol = R0 + lr;
        if (grow < N && gcol < M) {
          const float w = stage[ci * 33 + lr];
          if (p.D) p.D[grow * p.ldd + gcol] = w;
          if (p.Db) p.Db[grow * p.lddb + gcol] = __builtin_bit_cast(uint16_t, (__bf16)w);
          ss += (double)w * (double)w;
        }
      }
      __syncthreads();
    }
  }
  return ss;
}

template <int NW>
__device__ __forceinline__ void partial_at(const GemmLpArgs& p, double ss, double* red, int64_t u) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
  if (lane == 0) red[wave] = ss;
  __syncthreads();
  if (threadIdx.x == 0 && p.partial) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += red[w];
    p.partial[u] = t;
  }
}

template <int BM, int BK, bool VEC, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN) __attribute__((amdgpu_waves_per_eu(2)))
gemm_bf16_sym_kernel(GemmLpArgs p, int T, int dp, int splits, float* scratch) {
  constexpr int NT = 64 * WGM * WGN, NW = WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BM / WGN;
  constexpr int FM = WTM / 32, FN = WTN / 32;
  constexpr int S = BK + 8;
  constexpr int XV = (BM * BK / 8) / NT;
  static_assert(XV >= 1 && XV * NT == BM * BK / 8, "slab / thread mismatch");
  // X and Y slabs (two buffers each); the mirror stage of the epilogue
  // reuses the X slabs once the K loop is done.
  __shared__ __attribute__((aligned(16))) __bf16 Xs[2][BM * S];
  __shared__ __attribute__((aligned(16))) __bf16 Ys[2][BM * S];
  __shared__ double red[NW];
  static_assert(sizeof(Xs) >= NW * kStage * sizeof(float), "stage does not fit");

  const __bf16* X = static_cast<const __bf16*>(p.X);
  const __bf16* Y = static_cast<const __bf16*>(p.Y);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  const int lr = lane & 31, lk = lane >> 5;
  const int64_t M = p.M, N = p.N, K = p.K;
  const int nk = (int)((K + BK - 1) / BK);

  // Whole tile, or K-slice q of tail tile u.
  const bool tail = (int)blockIdx.x >= dp;
  int u, kt0, kt1;
  if (!tail) {
    u = blockIdx.x;
    kt0 = 0;
    kt1 = nk;
  } else {
    const int t = blockIdx.x - dp, q = t % splits;
    u = dp + t / splits;
    kt0 = (int)((int64_t)q * nk / splits);
    kt1 = (int)((int64_t)(q + 1) * nk / splits);
  }
  int tm, tn;
  sym_tile_lp(u, T, tm, tn);
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BM;
  uint4 xr[XV], yr[XV];

  auto load_one = [&](const __bf16* base, int64_t ld, int64_t r0, int64_t rmax, int64_t k0,
                      int v) -> uint4 {
    const int idx = tid + NT * v;
    const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
    const int64_t gr = r0 + row, gk = k0 + c;
    uint4 val = make_uint4(0u, 0u, 0u, 0u);
    if (gr < rmax) {
      const __bf16* src = base + gr * ld + gk;
      if (VEC && gk + 7 < K) {
        val = *reinterpret_cast<const uint4*>(src);
      } else {
        unsigned short tmp[8];
        const unsigned short* s16 = reinterpret_cast<const unsigned short*>(src);
#pragma unroll
        for (int e = 0; e < 8; ++e) tmp[e] = (gk + e < K) ? s16[e] : (unsigned short)0;
        val.x = tmp[0] | ((unsigned)tmp[1] << 16);
        val.y = tmp[2] | ((unsigned)tmp[3] << 16);
        val.z = tmp[4] | ((unsigned)tmp[5] << 16);
        val.w = tmp[6] | ((unsigned)tmp[7] << 16);
      }
    }
    return val;
  };
  const bool interior = VEC && (m0 + BM <= M) && (n0 + BM <= N);
  auto load = [&](int64_t k0) {
    if (interior && k0 + BK <= K) {
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int idx = tid + NT * v;
        const int64_t row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
        xr[v] = *reinterpret_cast<const uint4*>(X + (m0 + row) * p.ldx + k0 + c);
        yr[v] = *reinterpret_cast<const uint4*>(Y + (n0 + row) * p.ldy + k0 + c);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      xr[v] = load_one(X, p.ldx, m0, M, k0, v);
      yr[v] = load_one(Y, p.ldy, n0, N, k0, v);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 8), c = (idx % (BK / 8)) * 8;
      *reinterpret_cast<uint4*>(&Xs[buf][row * S + c]) = xr[v];
      *reinterpret_cast<uint4*>(&Ys[buf][row * S + c]) = yr[v];
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};

  if (kt0 < kt1) load((int64_t)kt0 * BK);
  for (int kt = kt0; kt < kt1; ++kt) {
    const int buf = kt & 1;
    store(buf);
    __syncthreads();
    if (kt + 1 < kt1) load((int64_t)(kt + 1) * BK);
    const __bf16* xs = &Xs[buf][(wm * WTM + lr) * S + 8 * lk];
    const __bf16* ys = &Ys[buf][(wn * WTN + lr) * S + 8 * lk];
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const bf16x8*>(xs + i * 32 * S + ks);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = *reinterpret_cast<const bf16x8*>(ys + j * 32 * S + ks);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __builtin_amdgcn_iglp_opt(1);
    if (NSR_LP_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }

  if (tail) {
    // Raw slice in accumulator order: consecutive lanes, consecutive floats.
    float* dst = scratch + (int64_t)(blockIdx.x - dp) * BM * BM +
                 (int64_t)wave * FM * FN * 1024 + lane;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) dst[((i * FN + j) * 16 + r) * 64] = acc[i][j][r];
    return;
  }
  __syncthreads();   // every wave is done reading the slabs the stage reuses
  float* stage = reinterpret_cast<float*>(&Xs[0][0]) + wave * kStage;
  const double ss = sym_epilogue<BM, WGM, WGN>(p, tm, tn, acc, stage);
  partial_at<NW>(p, ss, red, u);
}

// Finishes the tail tiles: workgroup t sums the `splits` slices of tail
// tile dp + t in slice order.
template <int BM, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
gemm_bf16_sym_fixup(GemmLpArgs p, int T, int dp, int splits, const float* scratch) {
  constexpr int NW = WGM * WGN, FM = BM / WGM / 32, FN = BM / WGN / 32;
  __shared__ float stage_all[NW * kStage];
  __shared__ double red[NW];
  const int t = blockIdx.x, u = dp + t;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x16{};
  for (int q = 0; q < splits; ++q) {
    const float* src = scratch + (int64_t)(t * splits + q) * BM * BM +
                       (int64_t)wave * FM * FN * 1024 + lane;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] += src[((i * FN + j) * 16 + r) * 64];
  }
  int tm, tn;
  sym_tile_lp(u, T, tm, tn);
  const double ss = sym_epilogue<BM, WGM, WGN>(p, tm, tn, acc, stage_all + wave * kStage);
  partial_at<NW>(p, ss, red, u);
}

bool big_tiles(int64_t m, int64_t n) { return ((m + 127) / 128) * ((n + 127) / 128) >= 256; }

}  // namespace

// Per-tile partial sums of any tile choice (64 x 64 tiles give the most).
int64_t gemm_lp_partials(int64_t m, int64_t n) { return ((m + 63) / 64) * ((n + 63) / 64); }

int64_t launch_gemm_f32_nn(const GemmLpArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return 0;
  const bool vec = ((a.ldx & 3) == 0) && ((a.ldy & 3) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Y) & 15) == 0);
  const int tc = tile_choice(kTileF32, a.M, a.N);
  // 256 x 256 tiles (LDS DMA) by the rule once they fill the CUs.
  // (The DMA sources are 32-bit byte offsets within 256 rows of X and 32 of Y.)
  const bool dma = NSR_F32_DMA && vec && (a.K % kF32DmaBK) == 0 && (a.N % 4) == 0 &&
                   (a.ldx % 4) == 0 && (a.ldy % 4) == 0 && a.ldx < (1 << 22) &&
                   a.ldy < (1 << 24);
  const bool huge = dma && (tc ? tc == 256 : ((a.M + 255) / 256) * ((a.N + 255) / 256) >= device_cus());
  const bool big = !huge && (tc ? tc == 128 || tc == 256 : big_tiles(a.M, a.N));
  const int bm = huge ? 256 : (big ? 128 : 64);
  const int tiles_m = (int)((a.M + bm - 1) / bm), tiles_n = (int)((a.N + bm - 1) / bm);
  dim3 grid((unsigned)((int64_t)tiles_m * tiles_n)), block(256);
  if (huge) {
    hipLaunchKernelGGL(gemm_f32_nn_dma_kernel, grid, dim3(512), 0, st, a, tiles_m, tiles_n);
  } else if (big) {
    // LDS-DMA K loop where its requirements hold (the DMA sources are 32-bit
    // byte offsets within 128 rows of X and 32 of Y).
    if (NSR_F32_DMA128 && vec && (a.K % 32) == 0 && (a.N % 4) == 0 && (a.ldx % 4) == 0 &&
        (a.ldy % 4) == 0 && a.ldx < (1 << 22) && a.ldy < (1 << 24))
      hipLaunchKernelGGL((gemm_f32_nn_kernel<128, 128, 32, true, true>), grid, block, 0, st, a,
                         tiles_m, tiles_n);
    else if (vec) hipLaunchKernelGGL((gemm_f32_nn_kernel<128, 128, 32, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_f32_nn_kernel<128, 128, 32, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  } else {
    if (vec) hipLaunchKernelGGL((gemm_f32_nn_kernel<64, 64, 32, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_f32_nn_kernel<64, 64, 32, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  }
  if (hipGetLastError() != hipSuccess) return -1;
  return a.partial ? (int64_t)tiles_m * tiles_n : 0;
}

int64_t launch_gemm_bf16_nt(const GemmLpArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return 0;
  const bool vec = ((a.ldx & 7) == 0) && ((a.ldy & 7) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Y) & 15) == 0);
  const int tc = tile_choice(kTileBf16, a.M, a.N);
  const bool huge = tc ? tc == 256 : NSR_BF16_HUGE && ((a.M + 255) / 256) * ((a.N + 255) / 256) >= 256;
  const bool big = tc ? tc == 128 : big_tiles(a.M, a.N);
  const int bm = huge ? 256 : (big ? 128 : 64);
  const int tiles_m = (int)((a.M + bm - 1) / bm), tiles_n = (int)((a.N + bm - 1) / bm);
  dim3 grid((unsigned)((int64_t)tiles_m * tiles_n)), block(256);
  if (huge) {
    // 256 x 256 tiles, eight waves of 128 x 64: half the L2 -> LDS bytes per
    // flop of the 128 x 128 tile, which saturates the L2.
    dim3 block8(512);
    const bool dma = NSR_BF16_DMA && vec && (a.K % kDmaBK) == 0 && (a.ldx % 8) == 0 &&
                     (a.ldy % 8) == 0;
    if (dma && (a.K % 64) == 0)
      hipLaunchKernelGGL((gemm_bf16_nt_dma_kernel<256, 2, 64>), grid, block8, 0, st, a, tiles_m,
                         tiles_n);
    else if (dma)
      hipLaunchKernelGGL((gemm_bf16_nt_dma_kernel<256, 4, 32>), grid, block8, 0, st, a, tiles_m,
                         tiles_n);
    else if (vec)
      hipLaunchKernelGGL((gemm_bf16_nt_kernel<256, 256, NSR_BF16_HUGE_BK, true, 2, 4>), grid,
                         block8, 0, st, a, tiles_m, tiles_n);
    else
      hipLaunchKernelGGL((gemm_bf16_nt_kernel<256, 256, NSR_BF16_HUGE_BK, false, 2, 4>), grid,
                         block8, 0, st, a, tiles_m, tiles_n);
  } else if (big) {
    const bool dma = NSR_BF16_DMA128 && vec && (a.K % kDmaBK) == 0 && (a.ldx % 8) == 0 &&
                     (a.ldy % 8) == 0;
    if (dma && (a.K % 64) == 0)
      hipLaunchKernelGGL((gemm_bf16_nt_dma_kernel<128, 2, 64, 128>), grid, block, 0, st, a,
                         tiles_m, tiles_n);
    else if (dma)
      hipLaunchKernelGGL((gemm_bf16_nt_dma_kernel<128, 4, 32, 128>), grid, block, 0, st, a,
                         tiles_m, tiles_n);
    else if (vec) hipLaunchKernelGGL((gemm_bf16_nt_kernel<128, 128, 64, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_bf16_nt_kernel<128, 128, 64, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  } else {
    if (vec) hipLaunchKernelGGL((gemm_bf16_nt_kernel<64, 64, 64, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_bf16_nt_kernel<64, 64, 64, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  }
  if (hipGetLastError() != hipSuccess) return -1;
  return a.partial ? (int64_t)tiles_m * tiles_n : 0;
}

int64_t launch_absmax(const float* X, int64_t ld, int64_t rows, int64_t cols, float* part,
                      hipStream_t st) {
  if (rows <= 0 || cols <= 0) return 0;
  const bool vec = ((ld & 3) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  const int64_t nb = rows < kSplitMaxParts ? rows : kSplitMaxParts;
  hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)nb), dim3(256), 0, st, X, ld, rows, cols, vec,
                     part);
  return nb;
}

void launch_split_f16(const float* X, int64_t ld, int64_t rows, int64_t cols, const float* part,
                      int64_t nparts, bool trans, uint16_t* hi, uint16_t* lo, int64_t ldh,
                      float* exp_out, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  const bool vec = ((ld & 3) == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (trans) {
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL(split_trans_kernel, grid, dim3(256), 0, st, X, ld, rows, cols, vec, part,
                       nparts, hi, lo, ldh, exp_out);
  } else {
    const int64_t chunks = rows * ((cols + 7) / 8);
    int64_t nb = (chunks + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)nb), dim3(256), 0, st, X, ld, rows, cols,
                       vec, part, nparts, hi, lo, ldh, exp_out);
  }
}

int64_t launch_gemm_f16s_nt(const GemmLpArgs& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return 0;
  const bool vec = ((a.ldx & 7) == 0) && ((a.ldy & 7) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Y) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Xl) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Yl) & 15) == 0);
  const int tc = tile_choice(kTileF16s, a.M, a.N);
  const bool huge = tc ? tc == 256 : ((a.M + 255) / 256) * ((a.N + 255) / 256) >= 256;
  const bool big = tc ? tc == 128 : big_tiles(a.M, a.N);
  const int bm = huge ? 256 : (big ? 128 : 64);
  const int tiles_m = (int)((a.M + bm - 1) / bm), tiles_n = (int)((a.N + bm - 1) / bm);
  dim3 grid((unsigned)((int64_t)tiles_m * tiles_n)), block(256);
  if (huge) {
    dim3 block8(512);
    // (The DMA sources are 32-bit byte offsets within 256 rows of a plane.)
    const bool dma = NSR_F16S_DMA && vec && (a.K % kF16sDmaBK) == 0 && (a.ldx % 8) == 0 &&
                     (a.ldy % 8) == 0 && a.ldx < (1 << 23) && a.ldy < (1 << 23);
    if (dma) hipLaunchKernelGGL(gemm_f16s_nt_dma_kernel<256>, grid, block8, 0, st, a, tiles_m, tiles_n);
    else if (vec) hipLaunchKernelGGL((gemm_f16s_nt_kernel<256, 256, 32, true, 2, 4>), grid, block8, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_f16s_nt_kernel<256, 256, 32, false, 2, 4>), grid, block8, 0, st, a, tiles_m, tiles_n);
  } else if (big) {
    const bool dma = NSR_F16S_DMA && vec && (a.K % kF16sDmaBK) == 0 && (a.ldx % 8) == 0 &&
                     (a.ldy % 8) == 0 && a.ldx < (1 << 23) && a.ldy < (1 << 23);
    if (dma) hipLaunchKernelGGL(gemm_f16s_nt_dma_kernel<128>, grid, block, 0, st, a, tiles_m, tiles_n);
    else if (vec) hipLaunchKernelGGL((gemm_f16s_nt_kernel<128, 128, 32, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_f16s_nt_kernel<128, 128, 32, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  } else {
    if (vec) hipLaunchKernelGGL((gemm_f16s_nt_kernel<64, 64, 32, true>), grid, block, 0, st, a, tiles_m, tiles_n);
    else hipLaunchKernelGGL((gemm_f16s_nt_kernel<64, 64, 32, false>), grid, block, 0, st, a, tiles_m, tiles_n);
  }
  if (hipGetLastError() != hipSuccess) return -1;
  return a.partial ? (int64_t)tiles_m * tiles_n : 0;
}

// Symmetric product plan: 128 x 128 tiles (four waves, two workgroups per
// CU; the eight-wave 256 x 256 variant needs more than 256 registers for the
// mirror epilogue).  Whole rounds of upper tiles run as they are; a partial
// last round after at least one whole round is cut into K-slices that fill
// the resident slots.  Costs are in rounds of the full-output kernel's
// 256 x 256 tiles: a round of 128-tiles does half the work per CU at about
// 87% of the rate (measured on the full kernels), 0.575 of a round.  Used
// where it saves at least 10% over the full-output kernel: from N ~ 3000
// (at N = 4096: 0.62 against 1 round; at N = 8192: 2.36 against 4).
struct SymPlan {
  int T = 0, dp = 0, tail = 0, splits = 1;
  double cost = 0.0;
};

static SymPlan sym_plan(int64_t n, int64_t k) {
  SymPlan pl;
  pl.T = (int)((n + 127) / 128);
  const int64_t tiles = (int64_t)pl.T * (pl.T + 1) / 2;
  const int64_t slots = 2 * (int64_t)device_cus();
  const int64_t rounds = tiles / slots, rem = tiles % slots;
  const int nk = (int)((k + 63) / 64);
  pl.dp = (int)tiles;
  pl.cost = (double)rounds + (rem ? 1.0 : 0.0);
  if (rounds >= 1 && rem > 0) {
    int sp = (int)(slots / rem);
    if (sp > nk) sp = nk;
    if (sp >= 2) {
      pl.dp = (int)(tiles - rem);
      pl.tail = (int)rem;
      pl.splits = sp;
      pl.cost = (double)rounds + (double)rem / (double)slots + 0.05;
    }
  }
  pl.cost *= 0.575;
  return pl;
}

static double full_cost(int64_t n) {
  const int64_t cus = device_cus();
  const int64_t t256 = (n + 255) / 256, t128 = (n + 127) / 128;
  if (NSR_BF16_HUGE && t256 * t256 >= cus) return (double)((t256 * t256 + cus - 1) / cus);
  return 0.575 * (double)((t128 * t128 + 2 * cus - 1) / (2 * cus));
}

static bool sym_choose(int64_t n, int64_t k, SymPlan& pl) {
  if (k <= 0 || n < 1024) return false;
  pl = sym_plan(n, k);
  return pl.cost <= 0.9 * full_cost(n);
}

int64_t gemm_bf16_sym_scratch_floats(int64_t n, int64_t k) {
  SymPlan pl;
  if (!sym_choose(n, k, pl)) return 0;
  return (int64_t)pl.tail * pl.splits * 128 * 128;
}

int64_t launch_gemm_bf16_sym(const GemmLpArgs& a, float* scratch, int64_t scratch_floats,
                             hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return 0;
  SymPlan pl;
  if (a.M != a.N || !sym_choose(a.N, a.K, pl)) return -2;
  const int64_t need = (int64_t)pl.tail * pl.splits * 128 * 128;
  if (need > 0 && (!scratch || scratch_floats < need)) return -2;
  const bool vec = ((a.ldx & 7) == 0) && ((a.ldy & 7) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Y) & 15) == 0);
  const dim3 grid((unsigned)(pl.dp + pl.tail * pl.splits));
  if (vec)
    hipLaunchKernelGGL((gemm_bf16_sym_kernel<128, 64, true, 2, 2>), grid, dim3(256), 0, st, a,
                       pl.T, pl.dp, pl.splits, scratch);
  else
    hipLaunchKernelGGL((gemm_bf16_sym_kernel<128, 64, false, 2, 2>), grid, dim3(256), 0, st, a,
                       pl.T, pl.dp, pl.splits, scratch);
  if (pl.tail)
    hipLaunchKernelGGL((gemm_bf16_sym_fixup<128, 2, 2>), dim3(pl.tail), dim3(256), 0, st, a,
                       pl.T, pl.dp, pl.splits, (const float*)scratch);
  if (hipGetLastError() != hipSuccess) return -1;
  return a.partial ? (int64_t)pl.T * (pl.T + 1) / 2 : 0;
}

}  // namespace nsr
