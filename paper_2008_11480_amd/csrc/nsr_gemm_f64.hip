// Float64 MFMA GEMM for gfx950 with the solver's fused epilogue
//
//   D = diag * I + scale * (X Y) + E1 + E2        (row-major, float64)
//
// Every product of the Newton-Schulz step is one such GEMM: the residual
// F = I - A G (diag = 1, scale = -1; eqs. xa2 / fk1), the powers F^2 = F F,
// the identity-offset assembly C' = C + F^(2^i) + C F^(2^i) of the factor
// (I + C)(I + F^(2^i)) (Tables 1-2), and the G-side update G + G C (eq. ns).
// When asked, the epilogue also writes one partial sum of D^2 per tile, which
// a fixed-order reduction turns into ||F||_F.
//
// Design (CDNA4):
//  * v_mfma_f64_16x16x4_f64: a wave multiplies 16x4 by 4x16 and accumulates a
//    16x16 float64 block; lane l supplies X[i = l%16][k = l/16] and
//    Y[k = l/16][j = l%16] and holds D[l/16 + 4 r][l%16], r = 0..3
//    (accumulator element r strides the rows by 4).
//  * A workgroup of 4 waves owns a BM x BN output tile; each wave owns a
//    (BM/2) x (BN/2) quadrant = (BM/32) x (BN/32) MFMA blocks kept in
//    registers for the whole K loop.
//  * K is walked in slabs of BK.  Each slab of X (BM x BK) and Y (BK x BN)
//    goes from global memory into one of two LDS stages, either straight by
//    LDS DMA (global_load_lds_dwordx4; the 128 x 128 tiles and the 256 x 128
//    full-product kernel, where the operands allow it) or through registers
//    one slab ahead (16-byte loads, coalesced along rows), and is read back
//    as MFMA fragments; one barrier per slab.
//  * Tile order is XCD-aware: consecutive workgroup ids land on different
//    XCDs, so each XCD is given a contiguous run of a grouped (8 tile-rows)
//    order, keeping the X row panels and Y column panels it reuses in its own
//    L2.
#include <atomic>

#include "nsr.h"
#include "nsr_internal.h"

// Tuning knobs of the large-tile configuration (chosen by measurement):
// K-slab depth, number of LDS slab buffers (2: one barrier per slab; 1: two
// barriers per slab, half the LDS) and the occupancy target in waves per SIMD.
#ifndef NSR_F64_BIG_BK
#define NSR_F64_BIG_BK 16
#endif
#ifndef NSR_F64_BIG_NBUF
#define NSR_F64_BIG_NBUF 2
#endif
#ifndef NSR_F64_WAVES_PER_EU
#define NSR_F64_WAVES_PER_EU 2
#endif
// 1: raise the wave's issue priority while it runs the slab's MFMAs.
#ifndef NSR_F64_SETPRIO
#define NSR_F64_SETPRIO 1
#endif
// 1: full products of large outputs use the 256 x 128 LDS-DMA kernel.
#ifndef NSR_F64_DMA
#define NSR_F64_DMA 1
#endif
// 1: the 128 x 128 tiles take their K slabs by LDS DMA where the operands
// allow it.
#ifndef NSR_F64_DMA128
#define NSR_F64_DMA128 1
#endif
// Row padding (doubles) of the X and Y slabs in LDS.
#ifndef NSR_F64_XPAD
#define NSR_F64_XPAD 2
#endif
#ifndef NSR_F64_YPAD
#define NSR_F64_YPAD 2
#endif

namespace nsr {

typedef double f64x4 __attribute__((ext_vector_type(4)));

namespace {

// Consecutive workgroup ids land on different XCDs: give each XCD a
// contiguous run of the tile order (count divisible by 8), so the panels a
// run reuses stay in that XCD's L2.
__device__ __forceinline__ int xcd_perm(int bid, int count) {
  return (count & 7) == 0 ? (bid & 7) * (count >> 3) + (bid >> 3) : bid;
}

// Position u of the grouped tile order (8 tile-rows per group) -> tile.
__device__ __forceinline__ void group_tile(int u, int tiles_m, int tiles_n, int& tm, int& tn) {
  constexpr int GM = 8;
  const int group_size = GM * tiles_n;
  const int g = u / group_size;
  const int first_m = g * GM;
  const int gm = min(tiles_m - first_m, GM);
  const int r = u - g * group_size;
  tm = first_m + r % gm;
  tn = r / gm;
}

// Upper-triangular tile t (row-major over tm <= tn) of a T x T tile grid.
__device__ __forceinline__ void sym_tile(int t, int T, int& tm, int& tn) {
  int r = t, m = 0;
  while (r >= T - m) {
    r -= T - m;
    ++m;
  }
  tm = m;
  tn = m + r;
}

__device__ __forceinline__ void tile_at(bool sym, int u, int tiles_m, int tiles_n, int& tm,
                                        int& tn) {
  if (sym)
    sym_tile(u, tiles_m, tm, tn);
  else
    group_tile(u, tiles_m, tiles_n, tm, tn);
}

// Mirror of the symmetric-output element D[row][col] = v: D[col][row] (equal
// to v, or v msc[col] / msc[row] for a diagonally similar output).
__device__ __forceinline__ double mirror_value(const GemmF64Args& p, int64_t row, int64_t col,
                                               double v) {
  return p.msc ? v * (p.msc[col] / p.msc[row]) : v;
}

// Output element: scale acc + diag [row == col] + E1 + E2, with the addends
// loaded beforehand (0 where absent).
__device__ __forceinline__ double epi_value(const GemmF64Args& p, int64_t row, int64_t col,
                                            double acc, double e1, double e2) {
  double v = p.scale * acc;
  if (row == col) v += p.diag;
  if (p.E1) v += e1;
  if (p.E2) v += e2;
  return v;
}

// Addends of one 16 x 16 accumulator fragment (rows row0 + 4 r, column col).
// The epilogue loads the next fragment's addends before it stores the
// current one: loads and stores share one in-order completion counter, so a
// load issued after a store waits for that store, and loading per element
// would put a memory round trip on every element.
__device__ __forceinline__ void load_addends(const GemmF64Args& p, int64_t row0, int64_t col,
                                             double (&e1)[4], double (&e2)[4]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = row0 + 4 * r;
    const bool in = row < p.M && col < p.N;
    e1[r] = (p.E1 && in) ? p.E1[row * p.lde1 + col] : 0.0;
    e2[r] = (p.E2 && in) ? p.E2[row * p.lde2 + col] : 0.0;
  }
}

// Row permutation of the 16-byte chunks of a 128-byte X slab row in the DMA
// form of gemm_f64_kernel: rows R and R + 1 sit in opposite bank halves, and
// (R >> 1) & 7 spreads the 16 rows of an MFMA operand read over the chunks,
// so a read of one double per lane (16 rows x 4 k) touches every bank once
// per 32 lanes.
__device__ __forceinline__ int f64_rsw(int row) { return (row >> 1) & 7; }

// Grid: the first dp workgroups own whole tiles (positions 0..dp-1 of the
// tile order).  When splits > 0, the remaining tiles (the last, partial round)
// are cut along K into `splits` slices of `slabs` K-slabs; workgroup dp + q
// computes slice q % splits of tail tile q / splits and stores its raw
// accumulators in p.sk (gemm_f64_split_fixup finishes those tiles).
//
// DMA (128 x 128 tiles, BK = 16, two stages; K a multiple of 16, N even, even
// row strides, 16-byte aligned X and Y): the K slabs go from global memory
// straight into LDS with global_load_lds_dwordx4, slab kt + 1 issued in two
// parts during slab kt's first two MFMA steps, one barrier per slab.  X rows
// (128 B) keep chunk c at c ^ f64_rsw(row); Y rows (1 KB) put chunk c at
// c ^ 8 in odd k rows, so the two k rows a 32-lane read group touches use
// opposite bank halves.  The MFMA sequence and the accumulator layout are
// those of the register-staged loop (the results are the same bits), so the
// epilogue, the mirror and the split tail are shared.  Rows past M and
// columns past N of edge tiles read row M - 1 and the last two columns and
// feed only outputs that are not stored.
template <int BM, int BN, int BK, int NBUF, bool VEC, bool SYM, bool DMA = false>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(NSR_F64_WAVES_PER_EU)))
gemm_f64_kernel(GemmF64Args p, int tiles_m, int tiles_n, int dp, int splits, int slabs) {
  constexpr int NT = 256;
  constexpr int WTM = BM / 2;          // rows per wave
  constexpr int WTN = BN / 2;          // cols per wave
  constexpr int FM = WTM / 16;
  constexpr int FN = WTN / 16;
  constexpr int XS = BK + NSR_F64_XPAD;   // LDS row stride of the X slab (doubles)
  constexpr int YS = BN + NSR_F64_YPAD;   // LDS row stride of the Y slab
  constexpr int XV = (BM * BK / 2) / NT;   // double2 per thread, X slab
  constexpr int YV = (BK * BN / 2) / NT;   // double2 per thread, Y slab
  static_assert(XV >= 1 && YV >= 1, "tile too small for 256 threads");
  static_assert((BM * BK / 2) % NT == 0 && (BK * BN / 2) % NT == 0, "tile/thread mismatch");

  // One LDS arena: the K-slab buffers, reused after the K loop to stage the
  // transposed half-tiles of the mirrored write (symmetric output).
  constexpr int MAIN = NBUF * (BM * XS + BK * YS);
  constexpr int MS = BM + 1;                 // stride of the transposed staging
  constexpr int MIRROR = SYM ? WTN * MS : 0;
  constexpr int ARENA = MAIN > MIRROR ? MAIN : MIRROR;
  static_assert(!DMA || (BM == 128 && BN == 128 && BK == 16 && NBUF == 2 && VEC),
                "DMA form: 128 x 128 tiles, 16-deep slabs, two stages");
  static_assert(!DMA || MAIN * 8 >= 2 * (BM * BK + BK * BN) * 8, "DMA ring fits the arena");
  __shared__ __attribute__((aligned(1024))) double smem[ARENA];
  __shared__ double red[4];
  double (*Xs)[BM * XS] = reinterpret_cast<double (*)[BM * XS]>(smem);
  double (*Ys)[BK * YS] = reinterpret_cast<double (*)[BK * YS]>(smem + NBUF * BM * XS);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1;
  const int wn = wave & 1;
  // Symmetric output: only tiles with tm <= tn (tiles_m == tiles_n).
  const int bid = blockIdx.x;
  const bool tail = bid >= dp;
  const int tile_id = tail ? dp + (bid - dp) / splits : xcd_perm(bid, dp);
  int tm, tn;
  tile_at(SYM, tile_id, tiles_m, tiles_n, tm, tn);
  const int64_t m0 = (int64_t)tm * BM;
  const int64_t n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N, K = p.K;

  double2 xr[XV];
  double2 yr[YV];

  // Tiles whose rows and columns lie inside the matrix load full slabs with
  // unchecked 16-byte loads (a wave-uniform branch); edge tiles and the last,
  // partial K slab take the checked path.
  const bool interior = VEC && (m0 + BM <= M) && (n0 + BN <= N);
  auto load = [&](int64_t k0) {
    if (interior && k0 + BK <= K) {
#pragma unroll
      for (int v = 0; v < XV; ++v) {
        const int idx = tid + NT * v;
        xr[v] = *reinterpret_cast<const double2*>(p.X + (m0 + idx / (BK / 2)) * p.ldx + k0 +
                                                  (idx % (BK / 2)) * 2);
      }
#pragma unroll
      for (int v = 0; v < YV; ++v) {
        const int idx = tid + NT * v;
        yr[v] = *reinterpret_cast<const double2*>(p.Y + (k0 + idx / (BN / 2)) * p.ldy + n0 +
                                                  (idx % (BN / 2)) * 2);
      }
      return;
    }
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 2);
      const int c = (idx % (BK / 2)) * 2;
      const int64_t gm = m0 + row;
      const int64_t gk = k0 + c;
      double2 val = make_double2(0.0, 0.0);
      if (gm < M) {
        const double* src = p.X + gm * p.ldx + gk;
        if (VEC && gk + 1 < K) {
          val = *reinterpret_cast<const double2*>(src);
        } else {
          if (gk < K) val.x = src[0];
          if (gk + 1 < K) val.y = src[1];
        }
      }
      xr[v] = val;
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BN / 2);
      const int c = (idx % (BN / 2)) * 2;
      const int64_t gk = k0 + row;
      const int64_t gn = n0 + c;
      double2 val = make_double2(0.0, 0.0);
      if (gk < K) {
        const double* src = p.Y + gk * p.ldy + gn;
        if (VEC && gn + 1 < N) {
          val = *reinterpret_cast<const double2*>(src);
        } else {
          if (gn < N) val.x = src[0];
          if (gn + 1 < N) val.y = src[1];
        }
      }
      yr[v] = val;
    }
  };

  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < XV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BK / 2);
      const int c = (idx % (BK / 2)) * 2;
      if constexpr ((XS & 1) == 0) {
        *reinterpret_cast<double2*>(&Xs[buf][row * XS + c]) = xr[v];
      } else {
        Xs[buf][row * XS + c] = xr[v].x;
        Xs[buf][row * XS + c + 1] = xr[v].y;
      }
    }
#pragma unroll
    for (int v = 0; v < YV; ++v) {
      const int idx = tid + NT * v;
      const int row = idx / (BN / 2);
      const int c = (idx % (BN / 2)) * 2;
      if constexpr ((YS & 1) == 0) {
        *reinterpret_cast<double2*>(&Ys[buf][row * YS + c]) = yr[v];
      } else {
        Ys[buf][row * YS + c] = yr[v].x;
        Ys[buf][row * YS + c + 1] = yr[v].y;
      }
    }
  };

  f64x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  int kt0 = 0, kt1 = (int)((K + BK - 1) / BK);
  if (tail) {
    kt0 = ((bid - dp) % splits) * slabs;
    kt1 = min(kt1, kt0 + slabs);
  }
  const int lr = lane & 15;
  const int lk = lane >> 4;
  if constexpr (DMA) {
    constexpr int XB = BM * BK * 8;          // 128 rows of 128 B
    constexpr int SB = XB + BK * BN * 8;     // + 16 rows of 1 KB
    const uint32_t ring_lds = lds_addr(smem);
    const unsigned char* ring = reinterpret_cast<const unsigned char*>(smem);
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // DMA sources as byte offsets from the slab's wave-uniform base: X
    // instruction u of this wave covers tile rows (4 u + wave) 8 .. + 7, Y
    // instruction u the slab row k = 4 u + wave.
    uint32_t xoff[4], yoff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int row = (4 * u + wv) * 8 + (lane >> 3);
      const int c = (lane & 7) ^ f64_rsw(row);
      const int64_t g = (m0 + row < M ? m0 + row : M - 1) - m0;
      xoff[u] = (uint32_t)((g * p.ldx + 2 * c) * 8);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = 4 * u + wv;
      const int64_t col = n0 + 2 * (lane ^ ((k & 1) << 3));
      yoff[u] = (uint32_t)(((int64_t)k * p.ldy + (col < N ? col : N - 2) - n0) * 8);
    }
    const double* xbase = p.X + m0 * p.ldx;
    const double* ybase = p.Y + n0;
    // Part h of slab kt: X and Y instructions 2 h and 2 h + 1.
    auto issue_part = [&](int kt, int h) {
      const uint32_t st = ring_lds + (uint32_t)((kt & 1) * SB);
      const double* xb = xbase + (int64_t)kt * BK;
      const double* yb = ybase + (int64_t)kt * BK * p.ldy;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int u = 2 * h + v;
        lds_dma16s(xb, xoff[u], st + (uint32_t)((4 * u + wv) * 1024));
        lds_dma16s(yb, yoff[u], st + (uint32_t)(XB + (4 * u + wv) * 1024));
      }
    };
    // Operand byte offsets within a stage for MFMA step t (k = 4 t + lk):
    // A X[wm 64 + 16 i + lr][k] at offa[t] + 2048 i, B Y[k][wn 64 + 16 j + lr]
    // at offb[j] + 4096 t.
    const int sw = f64_rsw(lr);   // = f64_rsw of every row this lane reads
    int offa[4], offb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      offa[t] = (wm * WTM + lr) * 128 + (((2 * t + (lk >> 1)) ^ sw) * 16) + (lk & 1) * 8;
#pragma unroll
    for (int j = 0; j < FN; ++j)
      offb[j] = XB + lk * 1024 +
                (((wn * WTN + 16 * j + lr) >> 1) ^ ((lk & 1) << 3)) * 16 + (lr & 1) * 8;
    auto read_ops = [&](int kt, int t, double (&a)[FM], double (&b)[FN]) {
      const unsigned char* stage = ring + (kt & 1) * SB;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const double*>(stage + offa[t] + 2048 * i);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        b[j] = *reinterpret_cast<const double*>(stage + offb[j] + 4096 * t);
    };
    double fa[2][FM], fb[2][FN];
    if (kt0 < kt1) {
      issue_part(kt0, 0);
      issue_part(kt0, 1);
      dma_wait_barrier<0>();
      read_ops(kt0, 0, fa[0], fb[0]);
    }
    if (NSR_F64_SETPRIO) __builtin_amdgcn_s_setprio(1);
    for (int kt = kt0; kt < kt1; ++kt) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (t < 3) {
          read_ops(kt, t + 1, fa[(t + 1) & 1], fb[(t + 1) & 1]);
        } else {
          // Slab kt + 1 has landed and every wave holds its slab-kt operands;
          // the reads follow on every path (after the last slab they read a
          // stage and go unused) so the compiler's LDS wait before this
          // step's MFMAs does not count them.
          dma_wait_barrier<0>();
          read_ops(kt + 1, 0, fa[0], fb[0]);
        }
        if (t < 2 && kt + 1 < kt1) issue_part(kt + 1, t);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[t & 1][i], fb[t & 1][j], acc[i][j],
                                                             0, 0, 0);
        // Each step's region: the next step's LDS reads first, then its MFMAs.
        __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    if (NSR_F64_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }
  if (!DMA && kt0 < kt1) load((int64_t)kt0 * BK);
  for (int kt = kt0; kt < kt1 && !DMA; ++kt) {
    const int buf = (NBUF == 2) ? (kt & 1) : 0;
    if (NBUF == 1 && kt > kt0) __syncthreads();   // everyone done reading the slab
    store(buf);
    __syncthreads();
    if (kt + 1 < kt1) load((int64_t)(kt + 1) * BK);
    const double* xs = &Xs[buf][(wm * WTM + lr) * XS + lk];
    const double* ys = &Ys[buf][lk * YS + wn * WTN + lr];
    if (NSR_F64_SETPRIO) __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = xs[i * 16 * XS + ks];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = ys[ks * YS + j * 16];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (NSR_F64_SETPRIO) __builtin_amdgcn_s_setprio(0);
  }

  if (tail) {
    // Raw K-slice of a tail tile, in accumulator order: consecutive lanes
    // store consecutive doubles.
    double* dst = p.sk + (size_t)(bid - dp) * (BM * BN) + lane;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[((wave * FM + i) * FN + j) * 256 + r * 64] = acc[i][j][r];
    return;
  }

  // Epilogue: D = diag I + scale acc + E1 + E2, optional sum of D^2.  With a
  // symmetric output a diagonal tile writes its upper triangle and mirrors it
  // element-wise; an off-diagonal tile writes itself and (below) its
  // transpose through LDS.
  double ss = 0.0;
  const bool diag_tile = SYM && (tm == tn);
  double e1[2][4], e2[2][4];
  load_addends(p, m0 + wm * WTM + lk, n0 + wn * WTN + lr, e1[0], e2[0]);
#pragma unroll
  for (int i = 0; i < FM; ++i) {
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int f = i * FN + j;
      if (f + 1 < FM * FN)
        load_addends(p, m0 + wm * WTM + ((f + 1) / FN) * 16 + lk,
                     n0 + wn * WTN + ((f + 1) % FN) * 16 + lr, e1[(f + 1) & 1], e2[(f + 1) & 1]);
      const int64_t col = n0 + wn * WTN + j * 16 + lr;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm * WTM + i * 16 + lk + 4 * r;
        if (row < M && col < N) {
          const double v = epi_value(p, row, col, acc[i][j][r], e1[f & 1][r], e2[f & 1][r]);
          if (SYM) acc[i][j][r] = v;
          if (!diag_tile) {
            p.D[row * p.ldd + col] = v;
            if (SYM) {
              const double w = mirror_value(p, row, col, v);
              ss += v * v + w * w;
            } else {
              ss += v * v;
            }
          } else if (row <= col) {
            p.D[row * p.ldd + col] = v;
            double w = 0.0;
            if (row < col) {
              w = mirror_value(p, row, col, v);
              p.D[col * p.ldd + row] = w;
            }
            ss += v * v + w * w;
          }
        }
      }
    }
  }
  if (SYM && !diag_tile) {
    // Mirror D[n0.., m0..] = tile^T, one column half (wn) at a time.
    double* S = smem;
    __syncthreads();  // K-loop reads of the arena are done
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (wn == half) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              S[(j * 16 + lr) * MS + wm * WTM + i * 16 + lk + 4 * r] = acc[i][j][r];
      }
      __syncthreads();
      for (int idx = tid; idx < WTN * BM; idx += NT) {
        const int c = idx / BM, rr = idx % BM;
        const int64_t grow = n0 + half * WTN + c, gcol = m0 + rr;
        if (grow < N && gcol < M)
          p.D[grow * p.ldd + gcol] = mirror_value(p, gcol, grow, S[c * MS + rr]);
      }
      __syncthreads();
    }
  }
  if (p.partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) p.partial[tile_id] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Finishes the split tail tiles: sums the K-slices of each tile in a fixed
// order, applies the epilogue and writes the tile (and its mirror).  One
// workgroup per 16-row MFMA strip of a wave quadrant (16 x BN/2 outputs);
// thread t plays lane t % 64 of MFMA column block t / 64, so the slices are
// read in the order the main kernel stored them.  Partial sums of D^2 go to
// p.partial[dp + blockIdx.x].
template <int BM, int BN, bool SYM>
__global__ void __launch_bounds__(256)
gemm_f64_split_fixup(GemmF64Args p, int tiles_m, int tiles_n, int dp, int splits) {
  constexpr int WTM = BM / 2, WTN = BN / 2, FM = WTM / 16, FN = WTN / 16;
  static_assert(FN * 64 == 256, "one thread per lane and MFMA column block");
  constexpr int TS = BM * BN;
  constexpr int SS = 17;
  __shared__ double S[SYM ? WTN * SS : 1];
  __shared__ double red[4];
  const int b = blockIdx.x;
  const int jt = b / (4 * FM);
  const int wave = (b / FM) % 4;
  const int i = b % FM;
  const int wm = wave >> 1, wn = wave & 1;
  int tm, tn;
  tile_at(SYM, dp + jt, tiles_m, tiles_n, tm, tn);
  const int tid = threadIdx.x, lane = tid & 63, jj = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int64_t M = p.M, N = p.N;
  const bool diag_tile = SYM && (tm == tn);
  const double* src = p.sk + (size_t)jt * splits * TS + ((wave * FM + i) * FN + jj) * 256 + lane;
  // Sum the K-slices in slice order (fixed, deterministic); four rows and
  // four slices per iteration keep 16 loads in flight.
  double acc4[4] = {0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 4 <= splits; q += 4) {
    double v[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) v[u][r] = src[(size_t)(q + u) * TS + r * 64];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc4[r] += v[u][r];
  }
  for (; q < splits; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc4[r] += src[(size_t)q * TS + r * 64];
  double ss = 0.0;
  double e1[4], e2[4];
  load_addends(p, m0 + wm * WTM + i * 16 + lk, n0 + wn * WTN + jj * 16 + lr, e1, e2);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double a = acc4[r];
    const int64_t row = m0 + wm * WTM + i * 16 + lk + 4 * r;
    const int64_t col = n0 + wn * WTN + jj * 16 + lr;
    if (row < M && col < N) {
      const double v = epi_value(p, row, col, a, e1[r], e2[r]);
      if (SYM) S[(jj * 16 + lr) * SS + lk + 4 * r] = v;
      if (!diag_tile) {
        p.D[row * p.ldd + col] = v;
        if (SYM) {
          const double w = mirror_value(p, row, col, v);
          ss += v * v + w * w;
        } else {
          ss += v * v;
        }
      } else if (row <= col) {
        p.D[row * p.ldd + col] = v;
        double w = 0.0;
        if (row < col) {
          w = mirror_value(p, row, col, v);
          p.D[col * p.ldd + row] = w;
        }
        ss += v * v + w * w;
      }
    }
  }
  if (SYM && !diag_tile) {
    __syncthreads();
    for (int idx = tid; idx < WTN * 16; idx += 256) {
      const int c = idx >> 4, rr = idx & 15;
      const int64_t grow = n0 + wn * WTN + c, gcol = m0 + wm * WTM + i * 16 + rr;
      if (grow < N && gcol < M)
        p.D[grow * p.ldd + gcol] = mirror_value(p, gcol, grow, S[c * SS + rr]);
    }
  }
  if (p.partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[tid >> 6] = ss;
    __syncthreads();
    if (tid == 0) p.partial[dp + b] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Full (not symmetric-output) products of large outputs: 256 x 128 tiles fed
// by LDS DMA, eight waves of 64 x 64 (one workgroup per CU, two waves per
// SIMD), K in 16-deep slabs that global_load_lds_dwordx4 writes into two
// LDS stages (an X slab: 256 rows of 128 B; a Y slab: 16 rows of 1 KB).
// One 16-byte read gives a lane the A operands of two MFMA steps: in
// k-group g (8 k) lane (r, q) = (lane % 16, lane / 16) holds
// X[row][8 g + 2 q + j] for step j, so its B operand in that step is
// Y[8 g + 2 q + j][col]; one 16-byte read of a Y row gives the B operands of
// two fragments (fragment jj of a wave's 32-column half takes the columns
// 2 r + jj), so after the K loop a lane holds two adjacent columns of each
// output row it owns and the epilogue moves them as one 16-byte access where
// the output allows.  X rows put chunk c at c ^ f64_xsw(R) (R mod 16 decides
// which bank half and window a lane of a 16-lane read group hits); the B
// reads need no permutation.  Requires K a multiple of 16, N even, even row
// strides and 16-byte aligned operands; rows past M and columns past N of
// edge tiles read row M - 1 and the last two columns instead and feed only
// outputs that are not stored.
constexpr int kF64DmaBK = 16;

__device__ __forceinline__ int f64_xsw(int row) { return (row & 2) | ((row >> 1) & 4); }

typedef double f64x2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2)))
gemm_f64_nn_dma_kernel(GemmF64Args p, int tiles_m, int tiles_n) {
  constexpr int BM = 256, BN = 128, BK = kF64DmaBK, NW = 8, NST = 2;
  constexpr int WTM = 64, WTN = 64, FM = WTM / 16, FN = WTN / 16;
  constexpr int XBYTES = BM * BK * 8;            // 256 rows of 128 B
  constexpr int SBYTES = XBYTES + BK * BN * 8;   // + 16 rows of 1 KB
  constexpr int XI = BM / 8 / NW, YI = BK / NW;  // DMA instructions per wave and slab
  static_assert(XI == 4 && YI == 2 && BN == 128, "DMA split");
  __shared__ __attribute__((aligned(1024))) unsigned char ring[NST * SBYTES];
  __shared__ double red[NW];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  int tm, tn;
  group_tile(xcd_perm(blockIdx.x, tiles_m * tiles_n), tiles_m, tiles_n, tm, tn);
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
    const int c = (lane & 7) ^ f64_xsw(row);
    const int64_t g = (m0 + row < M ? m0 + row : M - 1) - m0;
    xoff[u] = (uint32_t)((g * p.ldx + 2 * c) * 8);
  }
#pragma unroll
  for (int u = 0; u < YI; ++u) {
    const int k = u * NW + wave;
    const int64_t col = n0 + 2 * lane;
    yoff[u] = (uint32_t)(((int64_t)k * p.ldy + (col < N ? col : N - 2) - n0) * 8);
  }
  const double* xbase = p.X + m0 * p.ldx;
  const double* ybase = p.Y + n0;
  // Part h of slab kt's DMA: X instructions 2 h, 2 h + 1 and Y instruction h.
  auto issue_part = [&](int kt, int h) {
    const uint32_t st = ring_lds + (uint32_t)((kt % NST) * SBYTES);
    const double* xb = xbase + (int64_t)kt * BK;
#pragma unroll
    for (int v = 0; v < 2; ++v)
      lds_dma16s(xb, xoff[2 * h + v], st + (uint32_t)(((2 * h + v) * NW + wave) * 1024));
    lds_dma16s(ybase + (int64_t)kt * BK * p.ldy, yoff[h],
               st + (uint32_t)(XBYTES + (h * NW + wave) * 1024));
  };

  // Operand byte offsets within a stage.  A, k-group g, fragment i (+ 2048 i):
  // row wm 64 + r, chunk 4 g + q.  B, half h of the wave's columns, step j of
  // group g (+ 256 h + 1024 (8 g + j)): row 2 q, columns wn 64 + 2 r, + 1.
  const int r = lane & 15, q = lane >> 4;
  int offa[2];
#pragma unroll
  for (int g = 0; g < 2; ++g) offa[g] = (wm * WTM + r) * 128 + (((4 * g + q) ^ f64_xsw(r)) * 16);
  const int offb = XBYTES + q * 2048 + wn * 512 + 16 * r;
  auto read_a = [&](int kt, int g, f64x2 (&a)[FM]) {
    const unsigned char* stage = ring + (kt % NST) * SBYTES;
#pragma unroll
    for (int i = 0; i < FM; ++i) a[i] = *reinterpret_cast<const f64x2*>(stage + offa[g] + i * 2048);
  };
  auto read_b = [&](int kt, int t, double (&b)[FN]) {   // step t = 2 g + j of the slab
    const unsigned char* stage = ring + (kt % NST) * SBYTES + (8 * (t >> 1) + (t & 1)) * 1024;
#pragma unroll
    for (int h = 0; h < FN / 2; ++h) {
      const f64x2 v = *reinterpret_cast<const f64x2*>(stage + offb + h * 256);
      b[2 * h] = v[0];
      b[2 * h + 1] = v[1];
    }
  };

  f64x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  // A is read a k-group (two steps) ahead, B a step ahead.  Slab kt + 1's DMA
  // is issued in two parts over slab kt's first two steps into the stage slab
  // kt - 1 used; the barrier before slab kt's last step (every wave then
  // holds all its operands of slab kt) makes it visible and frees slab kt's
  // stage.
  const int nk = (int)(K / BK);
  f64x2 fa[2][FM];
  double fb[2][FN];
  if (nk > 0) {
    issue_part(0, 0);
    issue_part(0, 1);
    dma_wait_barrier<0>();
    read_a(0, 0, fa[0]);
    read_b(0, 0, fb[0]);
  }
  for (int kt = 0; kt < nk; ++kt) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t == 0) read_a(kt, 1, fa[1]);
      if (t < 3) {
        read_b(kt, t + 1, fb[(t + 1) & 1]);
      } else {
        // Also after the last slab (the reads are then unused): with the
        // reads on every path the compiler's LDS wait before this step's
        // MFMAs does not count them.
        dma_wait_barrier<0>();
        read_a(kt + 1, 0, fa[0]);
        read_b(kt + 1, 0, fb[0]);
      }
      if (t < 2 && kt + 1 < nk) issue_part(kt + 1, t);
      const int g = t >> 1, jstep = t & 1;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[g][i][jstep], fb[t & 1][j], acc[i][j],
                                                           0, 0, 0);
      // Each step's region: the next step's LDS reads first, then its MFMAs.
      __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  // Output unit u = (fragment row i, column half h, element e): the lane's
  // row wm 64 + 16 i + q + 4 e and columns wn 64 + 32 h + 2 r, + 1, the values
  // acc[i][2 h + jj][e].  Where every output and addend allows it the two
  // columns go as one 16-byte access; the addends of unit u + PD are loaded
  // before unit u's stores (loads and stores complete in issue order); units
  // by compile-time index (a run-time index would put acc in scratch).
  constexpr int PD = 4, NU = FM * (FN / 2) * 4;
  const bool vec = ((uintptr_t)p.D & 15) == 0 && (p.ldd & 1) == 0 &&
                   (!p.E1 || (((uintptr_t)p.E1 & 15) == 0 && (p.lde1 & 1) == 0)) &&
                   (!p.E2 || (((uintptr_t)p.E2 & 15) == 0 && (p.lde2 & 1) == 0));
  double ss = 0.0;
  f64x2 e1[PD + 1], e2[PD + 1];
  auto unit_row = [&](int u) { return m0 + wm * WTM + 16 * (u >> 3) + q + 4 * (u & 3); };
  auto unit_col = [&](int u) { return n0 + wn * WTN + 32 * ((u >> 2) & 1) + 2 * r; };
  auto load2 = [&](int u, f64x2& a1, f64x2& a2) {
    const int64_t row = unit_row(u), col = unit_col(u);
    a1 = f64x2{0.0, 0.0};
    a2 = a1;
    if (row >= M) return;
    if (vec && col + 1 < N) {
      if (p.E1) a1 = *reinterpret_cast<const f64x2*>(p.E1 + row * p.lde1 + col);
      if (p.E2) a2 = *reinterpret_cast<const f64x2*>(p.E2 + row * p.lde2 + col);
      return;
    }
#pragma unroll
    for (int jj = 0; jj < 2; ++jj)
      if (col + jj < N) {
        if (p.E1) a1[jj] = p.E1[row * p.lde1 + col + jj];
        if (p.E2) a2[jj] = p.E2[row * p.lde2 + col + jj];
      }
  };
  static_for<0, PD>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    load2(u, e1[u], e2[u]);
  });
  static_for<0, NU>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    if constexpr (u + PD < NU) load2(u + PD, e1[(u + PD) % (PD + 1)], e2[(u + PD) % (PD + 1)]);
    constexpr int i = u >> 3, h = (u >> 2) & 1, e = u & 3, b = u % (PD + 1);
    const int64_t row = unit_row(u), col = unit_col(u);
    if (row < M) {
      f64x2 v;
#pragma unroll
      for (int jj = 0; jj < 2; ++jj)
        v[jj] = epi_value(p, row, col + jj, acc[i][2 * h + jj][e], e1[b][jj], e2[b][jj]);
      if (vec && col + 1 < N) {
        *reinterpret_cast<f64x2*>(p.D + row * p.ldd + col) = v;
        ss += v[0] * v[0] + v[1] * v[1];
      } else {
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          if (col + jj < N) {
            p.D[row * p.ldd + col + jj] = v[jj];
            ss += v[jj] * v[jj];
          }
      }
    }
  });
  if (p.partial) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) t += red[w];
      p.partial[(int64_t)tm * tiles_n + tn] = t;
    }
  }
}

// How one product is cut into workgroups.
struct Plan {
  bool big = false;    // 128 x 128 tiles (else 64 x 64)
  int64_t nt = 0;      // output tiles
  int64_t dp = 0;      // tiles owned whole by one workgroup
  int splits = 0;      // K-slices per tail tile (0: no tail)
  int slabs = 0;       // K-slabs per slice
};

template <int BM, int BN, int BK, int NBUF>
int64_t launch_cfg(const GemmF64Args& a, const Plan& pl, hipStream_t st) {
  const int tiles_m = (int)((a.M + BM - 1) / BM);
  const int tiles_n = (int)((a.N + BN - 1) / BN);
  const bool vec = ((a.ldx & 1) == 0) && ((a.ldy & 1) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.X) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(a.Y) & 15) == 0);
  const int64_t tail = pl.splits > 0 ? pl.nt - pl.dp : 0;
  dim3 grid((unsigned)(pl.dp + tail * pl.splits)), block(256);
  const int dp = (int)pl.dp, splits = pl.splits, slabs = pl.slabs;
  // LDS-DMA K loop where its requirements hold (the DMA sources are 32-bit
  // byte offsets within 128 rows of X and 16 of Y).
  bool launched = false;
  if constexpr (BM == 128 && BN == 128 && BK == 16 && NBUF == 2) {
    if (NSR_F64_DMA128 && vec && (a.K % 16) == 0 && (a.N % 2) == 0 && a.ldx < (1 << 21) &&
        a.ldy < (1 << 24)) {
      if (a.sym)
        hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, true, true, true>), grid, block, 0,
                           st, a, tiles_m, tiles_n, dp, splits, slabs);
      else
        hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, true, false, true>), grid, block, 0,
                           st, a, tiles_m, tiles_n, dp, splits, slabs);
      launched = true;
    }
  }
  if (launched) {
  } else if (a.sym) {
    if (vec)
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, true, true>), grid, block, 0, st, a,
                         tiles_m, tiles_n, dp, splits, slabs);
    else
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, false, true>), grid, block, 0, st, a,
                         tiles_m, tiles_n, dp, splits, slabs);
  } else {
    if (vec)
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, true, false>), grid, block, 0, st, a,
                         tiles_m, tiles_n, dp, splits, slabs);
    else
      hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, NBUF, false, false>), grid, block, 0, st, a,
                         tiles_m, tiles_n, dp, splits, slabs);
  }
  if (hipGetLastError() != hipSuccess) return -1;
  int64_t fix_blocks = 0;
  if constexpr (BN == 128) {
    if (tail > 0) {
      fix_blocks = tail * 4 * (BM / 32);
      dim3 fgrid((unsigned)fix_blocks);
      if (a.sym)
        hipLaunchKernelGGL((gemm_f64_split_fixup<BM, BN, true>), fgrid, block, 0, st, a, tiles_m,
                           tiles_n, dp, splits);
      else
        hipLaunchKernelGGL((gemm_f64_split_fixup<BM, BN, false>), fgrid, block, 0, st, a, tiles_m,
                           tiles_n, dp, splits);
      if (hipGetLastError() != hipSuccess) return -1;
    }
  }
  return a.partial ? pl.dp + fix_blocks : 0;
}

// Tile shape: 128 x 128 (two workgroups per CU) or 64 x 64 (four per CU).
// Time ~ rounds of resident workgroups x time of one tile; a partial last
// round that fills at most half the slots (one workgroup per CU) costs about
// half a round (its tiles run with less contention), a fuller one a round,
// and a 64 x 64 tile takes 0.54 of a 128 x 128 one at the same K.  Fitted to
// the measured full / symmetric GEMMs at N = 2048, 4096, 8192 (N = 2048 full
// products with the DMA K loop: 0.270 ms on 256 tiles of 128, one per CU,
// against 0.301 ms on 64 x 64 tiles).  A third choice, given scratch: 128 x 128 tiles
// whose last, partial round is cut along K into as many slices as fill the
// resident slots (a tail of r tiles in S slots takes ~ S / r times less than
// a round), finished by a small reduction kernel.  NSR_F64_FORCE_TILE (128
// or 64) restricts the shape, NSR_F64_SPLIT=0 disables the split.
#ifndef NSR_F64_FORCE_TILE
#define NSR_F64_FORCE_TILE 0
#endif
#ifndef NSR_F64_SPLIT
#define NSR_F64_SPLIT 1
#endif
constexpr int64_t kBigTile = 128 * 128;

double eff_rounds(int64_t tiles, int64_t slots) {
  const int64_t full = tiles / slots, rem = tiles % slots;
  return (double)full + (rem == 0 ? 0.0 : (2 * rem > slots ? 1.0 : 0.5));
}

int64_t tile_count(int64_t m, int64_t n, int64_t b, bool sym) {
  const int64_t tm = (m + b - 1) / b, tn = (n + b - 1) / b;
  return sym ? tm * (tm + 1) / 2 : tm * tn;
}

Plan plan_f64(int64_t m, int64_t n, int64_t k, bool sym, int64_t sk_cap) {
  const int64_t cus = device_cus();
  const int64_t s128 = 2 * cus;
  const int64_t c128 = tile_count(m, n, 128, sym), c64 = tile_count(m, n, 64, sym);
  const int tc = tile_choice(kTileF64, m, n);          // the tile autotuner's choice
  const int force = tc ? tc : NSR_F64_FORCE_TILE;
  Plan pl;
  double cost = 0.0;
  if (force == 128 ||
      (force != 64 && eff_rounds(c128, s128) <= 0.54 * eff_rounds(c64, 4 * cus))) {
    pl.big = true;
    pl.nt = pl.dp = c128;
    cost = eff_rounds(c128, s128);
  } else {
    pl.nt = pl.dp = c64;
    cost = 0.54 * eff_rounds(c64, 4 * cus);
  }
  const int64_t rem = c128 % s128;
  if (NSR_F64_SPLIT && force != 64 && sk_cap > 0 && c128 > s128 && rem != 0) {
    const int64_t nk = (k + 15) / 16;
    int64_t sp = s128 / rem < nk ? s128 / rem : nk;
    if (sp >= 2) {
      const int64_t slabs = (nk + sp - 1) / sp;
      sp = (nk + slabs - 1) / slabs;
      const double c = (double)(c128 / s128) + (double)slabs / (double)nk + 0.02;
      if (rem * sp * kBigTile <= sk_cap && c < cost) {
        pl.big = true;
        pl.nt = c128;
        pl.dp = c128 - rem;
        pl.splits = (int)sp;
        pl.slabs = (int)slabs;
      }
    }
  }
  return pl;
}

}  // namespace

namespace {
// Tile choices of the tile autotuner (ns_tile_set), per GEMM family and
// bucket ceil(log2(max(m, n))); 0 = the library's rule.
constexpr int kTileBuckets = 24;
std::atomic<int> g_tiles[kTileFamilies][kTileBuckets];

int tile_bucket(int64_t d) {
  int b = 0;
  while (b + 1 < kTileBuckets && ((int64_t)1 << b) < d) ++b;
  return b;
}

// Every family has the tiles 64, 128 and 256 (float64: 256 x 128 for full
// products); 0 selects the fitted rule.
bool tile_valid(int /*family*/, int tile) {
  return tile == 0 || tile == 64 || tile == 128 || tile == 256;
}
}  // namespace

int tile_choice(int family, int64_t m, int64_t n) {
  if (family < 0 || family >= kTileFamilies) return 0;
  return g_tiles[family][tile_bucket(m > n ? m : n)].load(std::memory_order_relaxed);
}

int device_cus() {
  // Read and written by any host thread that plans a launch: atomic, and
  // every writer stores the same value.
  static std::atomic<int> cus{0};
  int c = cus.load(std::memory_order_relaxed);
  if (c == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      c = v;
    else
      c = 256;
    cus.store(c, std::memory_order_relaxed);
  }
  return c;
}

int64_t gemm_f64_partials(int64_t m, int64_t n, bool sym) {
  // whole tiles + 16 fixup strips per split tail tile, or the 64 x 64 grid
  const int64_t c128 = tile_count(m, n, 128, sym), c64 = tile_count(m, n, 64, sym);
  const int64_t s128 = 2 * device_cus();
  const int64_t bound128 = c128 > s128 ? c128 + 15 * (c128 % s128) : c128;
  return bound128 > c64 ? bound128 : c64;
}

size_t gemm_f64_split_bytes(int64_t m, int64_t n, int64_t k, bool sym) {
  if (m <= 0 || n <= 0 || k <= 0 || (sym && m != n)) return 0;
  const Plan pl = plan_f64(m, n, k, sym, INT64_MAX);
  return pl.splits > 0 ? (size_t)(pl.nt - pl.dp) * pl.splits * kBigTile * sizeof(double) : 0;
}

int64_t launch_gemm_f64(const GemmF64Args& a, hipStream_t st) {
  if (a.M <= 0 || a.N <= 0) return 0;
  if (a.sym && a.M != a.N) return -1;
  // Full products of outputs that fill the CUs with 256 x 128 tiles take the
  // LDS-DMA kernel where its requirements hold (the DMA sources are 32-bit
  // byte offsets within 256 rows of X and 16 of Y).
  const int tc = tile_choice(kTileF64, a.M, a.N);
  const bool dma = NSR_F64_DMA && !a.sym && (a.K % kF64DmaBK) == 0 && (a.N % 2) == 0 &&
                   (a.ldx % 2) == 0 && (a.ldy % 2) == 0 &&
                   (reinterpret_cast<uintptr_t>(a.X) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(a.Y) & 15) == 0 && a.ldx < (1 << 21) &&
                   a.ldy < (1 << 24);
  const int tiles_m = (int)((a.M + 255) / 256), tiles_n = (int)((a.N + 127) / 128);
  if (dma && (tc ? tc == 256 : (int64_t)tiles_m * tiles_n >= device_cus())) {
    hipLaunchKernelGGL(gemm_f64_nn_dma_kernel, dim3((unsigned)(tiles_m * tiles_n)), dim3(512), 0,
                       st, a, tiles_m, tiles_n);
    if (hipGetLastError() != hipSuccess) return -1;
    return a.partial ? (int64_t)tiles_m * tiles_n : 0;
  }
  const Plan pl = plan_f64(a.M, a.N, a.K, a.sym != 0, a.sk ? a.sk_cap : 0);
  if (pl.big) return launch_cfg<128, 128, NSR_F64_BIG_BK, NSR_F64_BIG_NBUF>(a, pl, st);
  return launch_cfg<64, 64, 16, 2>(a, pl, st);
}

}  // namespace nsr

extern "C" {

int ns_tile_set(int family, int log2_dim, int tile) {
  if (family < 0 || family >= nsr::kTileFamilies || log2_dim < 0 ||
      log2_dim >= nsr::kTileBuckets || !nsr::tile_valid(family, tile)) {
    nsr::ns_set_error("ns_tile_set: unknown family, bucket or tile");
    return NS_EINVAL;
  }
  nsr::g_tiles[family][log2_dim].store(tile, std::memory_order_relaxed);
  return NS_OK;
}

int ns_tile_get(int family, int log2_dim) {
  if (family < 0 || family >= nsr::kTileFamilies || log2_dim < 0 ||
      log2_dim >= nsr::kTileBuckets)
    return -1;
  return nsr::g_tiles[family][log2_dim].load(std::memory_order_relaxed);
}

}  // extern "C"
