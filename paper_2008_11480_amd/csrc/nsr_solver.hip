// Solver runtime behind the C ABI of include/nsr.h.
//
// Holds the iteration state in the caller's workspace, turns each Newton-Schulz
// step into a chain of fused GEMM launches (one per matrix-matrix product the
// paper counts), runs the coupled Richardson update, and applies the stop
// rules.  Kernels live in nsr_gemm_f64.hip and nsr_blas2.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "nsr.h"
#include "nsr_internal.h"

using namespace nsr;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace

namespace nsr {
void ns_set_error(const char* msg) { snprintf(g_err, sizeof(g_err), "%s", msg); }
}  // namespace nsr

namespace {

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(NS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

constexpr size_t kAlign = 256;
// Margin of the error-law floor test of the stop rule.
constexpr double kLawMargin = 1e3;
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t ld_for(int64_t n) { return (n + 31) / 32 * 32; }

// One n x n iterate: float64 storage (plain mode) or float32 storage with an
// optional bf16 copy (float32 / mixed modes; the copy feeds bf16 products).
struct Mat {
  double* d = nullptr;
  float* f = nullptr;
  uint16_t* b = nullptr;
};

// Matrices of the iteration.  Plain: G0 G1 F P0 P1 C0 C1 (7); composite adds
// L0 L1 Gam H (11).  In mixed mode F, P*, C*, Gam carry bf16 copies.
constexpr int kPlainMats = 7;
constexpr int kMaxLoops = 3;   // parallel power series of the general composite

// Matrices for a composite level (0: plain; 1: double Newton-Schulz, [sri]
// and the general composite with one loop: L0 L1 Gam H; each further loop of
// the general composite: T0 T1 Gamma).  bf16 copies (mixed mode): F, P*, C*
// and one Gamma per loop.
int level_mats(int level) { return kPlainMats + (level >= 1 ? 4 : 0) + 3 * (level > 1 ? level - 1 : 0); }
int level_shadows(int level) { return 5 + level; }

int64_t partial_capacity(int64_t n) {
  int64_t c = gemm_f64_partials(n, n, false);
  c = c > gemm_f64_partials(n, n, true) ? c : gemm_f64_partials(n, n, true);
  c = c > gemm_lp_partials(n, n) ? c : gemm_lp_partials(n, n);
  c = c > sumsq_partials(n) ? c : sumsq_partials(n);
  c = c > gemv_partials(n) ? c : gemv_partials(n);
  c = c > 1024 ? c : 1024;
  c = c > n ? c : n;  // row sums for the infinity norm
  return c;
}

size_t split_bytes(int64_t n) {
  const size_t a = gemm_f64_split_bytes(n, n, n, false), b = gemm_f64_split_bytes(n, n, n, true);
  return a > b ? a : b;
}

// Scratch of a split half-precision product (m x n x k): hi / lo planes of
// X (m x k) and of Y^T (n x k) with a leading dimension padded to 8 halves,
// the per-block maxima of both operands and their two scale exponents.
struct SplitPlanes {
  uint16_t *xh, *xl, *yh, *yl;
  float* part;   // 2 kSplitMaxParts
  float* exps;   // 2
  int64_t ldk;
};

int64_t split_ld(int64_t k) { return ((k > 0 ? k : 1) + 7) / 8 * 8; }

size_t split_scratch_bytes(int64_t m, int64_t n, int64_t k) {
  const int64_t ldk = split_ld(k);
  return 2 * align_up((size_t)m * ldk * 2, kAlign) + 2 * align_up((size_t)n * ldk * 2, kAlign) +
         align_up(2 * kSplitMaxParts * sizeof(float), kAlign) + align_up(2 * sizeof(float), kAlign);
}

SplitPlanes carve_split(char* p, int64_t m, int64_t n, int64_t k) {
  SplitPlanes sp{};
  sp.ldk = split_ld(k);
  auto take = [&](size_t bytes) {
    char* q = p;
    p += align_up(bytes, kAlign);
    return q;
  };
  sp.xh = reinterpret_cast<uint16_t*>(take((size_t)m * sp.ldk * 2));
  sp.xl = reinterpret_cast<uint16_t*>(take((size_t)m * sp.ldk * 2));
  sp.yh = reinterpret_cast<uint16_t*>(take((size_t)n * sp.ldk * 2));
  sp.yl = reinterpret_cast<uint16_t*>(take((size_t)n * sp.ldk * 2));
  sp.part = reinterpret_cast<float*>(take(2 * kSplitMaxParts * sizeof(float)));
  sp.exps = reinterpret_cast<float*>(take(2 * sizeof(float)));
  return sp;
}

// Split a rows x cols float32 matrix into hi / lo planes (transposed when
// trans: the planes are then cols x rows), exponent to exp_out[0].
void split_operand(const float* X, int64_t ld, int64_t rows, int64_t cols, bool trans,
                   uint16_t* hi, uint16_t* lo, int64_t ldh, float* part, float* exp_out,
                   hipStream_t st) {
  const int64_t np = launch_absmax(X, ld, rows, cols, part, st);
  launch_split_f16(X, ld, rows, cols, part, np, trans, hi, lo, ldh, exp_out, st);
}

size_t elem_bytes(int precision) { return precision == NS_PREC_FP64 ? 8 : 4; }

bool mixed_prec(int precision) {
  return precision == NS_PREC_MIXED_BF16 || precision == NS_PREC_MIXED_SPLIT;
}

// Split mode: the row-major planes of A (the residual's left operand, split
// once per ns_bind) and the scratch of one split product.
size_t split_mode_bytes(int64_t n) {
  return 2 * align_up((size_t)n * split_ld(n) * 2, kAlign) + align_up(sizeof(float), kAlign) +
         split_scratch_bytes(n, n, n);
}

size_t layout_bytes(int64_t n, int precision, int composite) {
  const int64_t ld = ld_for(n);
  const size_t nn = (size_t)n * ld;
  size_t bytes = 0;
  const int mats = level_mats(composite);
  bytes += (size_t)mats * align_up(nn * elem_bytes(precision), kAlign);
  if (precision != NS_PREC_FP64) bytes += align_up(nn * 4, kAlign);          // float32 A
  if (mixed_prec(precision))
    bytes += (size_t)level_shadows(composite) * align_up(nn * 2, kAlign);    // bf16 copies
  if (precision == NS_PREC_MIXED_SPLIT) bytes += split_mode_bytes(n);        // split planes
  bytes += 5 * align_up((size_t)n * sizeof(double), kAlign);                 // r, t, w0, w1, S
  bytes += align_up((size_t)partial_capacity(n) * sizeof(double), kAlign);   // partials
  bytes += align_up(16 * sizeof(double), kAlign);                            // scalars
  bytes += align_up((NS_HIST_F + NS_HIST_R) * sizeof(double), kAlign);       // device history
  if (precision == NS_PREC_FP64) bytes += align_up(split_bytes(n), kAlign);  // split-K scratch
  return bytes;
}

struct TimedLaunch {
  hipEvent_t beg, end;
  int kind;
  double flop;
};

// Kind of product: the residual I - A X, a power / assembly product of
// polynomials in F (bf16 in mixed mode), or a G-side / merge product.
enum Kind { K_RESID = 0, K_POWER = 1, K_APPLY = 2 };

}  // namespace

struct ns_solver {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int64_t ld = 0;
  int precision = NS_PREC_FP64;
  int composite_capable = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;

  Mat G[2];
  int gcur = 0;
  Mat F, P[2], C[2];
  Mat L[2];
  int lcur = 0;
  Mat Gam, H;
  Mat LT[kMaxLoops - 1][2], LG[kMaxLoops - 1];   // loops 2.. of the general composite
  Mat* loopT[kMaxLoops][2] = {};
  Mat* loopG[kMaxLoops] = {};
  int tcur[kMaxLoops] = {0, 0, 0};
  int gc_w = 0;                    // general composite: number of loops (0: not set)
  int gc_m[kMaxLoops] = {0, 0, 0}; // their orders m_i (x_i = m_i^k)
  bool gc_started = false;
  float* A32 = nullptr;
  uint16_t* Ah = nullptr;  // split mode: half-precision planes of A32
  uint16_t* Al = nullptr;
  float* aexp = nullptr;   // and their scale exponent
  SplitPlanes sp{};        // split mode: scratch of one split product
  double* r = nullptr;
  double* vt = nullptr;      // accelerator temporaries (eq. ttk1)
  double* vw[2] = {nullptr, nullptr};
  double* partial = nullptr;
  double* scal = nullptr;  // [0] alpha, [1] ||F||_F, [2] ||r||_2, [3] ||b||_2, [4] -min A_ii
  double* dhist = nullptr; // device history of a captured iteration: ||F_k||, then ||r||
  // Captured fixed-length Newton-Schulz phase (opts.graph): the executable
  // graph, the key it was captured for and the host state after it.
  hipGraphExec_t graph_exec = nullptr;
  struct GraphKey {
    int order, fact, p, w, k, precision, symmetric, diag_scale;
    const double *A, *b;
    double* theta;
    int64_t lda;
    bool operator==(const GraphKey& o) const {
      return order == o.order && fact == o.fact && p == o.p && w == o.w && k == o.k &&
             precision == o.precision && symmetric == o.symmetric &&
             diag_scale == o.diag_scale && A == o.A && b == o.b && theta == o.theta &&
             lda == o.lda;
    }
  } graph_key{};
  hipStream_t capture_stream = nullptr;
  int graph_gcur = 0;
  int64_t graph_mmm = 0;
  double graph_flop = 0.0;
  double* sdiag = nullptr; // S = diag(A) (NS_SCALE_DIAG)
  bool diag_scale = false; // G_0 = diag(A)^-1 instead of I / alpha
  double* sk = nullptr;    // split-K scratch of the float64 GEMM
  int64_t sk_cap = 0;      // doubles

  const double* A = nullptr;
  int64_t lda = 0;
  bool bound = false;
  bool scaled = false;
  bool g_implicit = true;  // G = I / alpha, not materialised
  bool dns_started = false;
  bool p0_is_f2 = false;   // P[0] holds F_k^2 (computed by the floor test)
  bool symmetric = true;   // products with symmetric output (upper tiles + mirror)
  double alpha = 0.0;
  int64_t mmm = 0;
  double flop = 0.0;       // algorithmic flop of the products since ns_init_scale

  bool timing = false;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
};

namespace {

hipEvent_t take_event(ns_solver* s) {
  if (s->pool_used == s->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->pool.push_back(e);
  }
  return s->pool[s->pool_used++];
}

bool is_f64(const ns_solver* s) { return s->precision == NS_PREC_FP64; }

// One fused GEMM D = diag I + scale X Y + E1 + E2 on the solver's stream.
// X == nullptr means A (the residual products).  Dispatch by precision:
// float64 MFMA; float32 MFMA; mixed: bf16 MFMA (X Y^T) for K_POWER products,
// float32 MFMA otherwise (split mode: the float32-class product of split
// half-precision operands).
int mm(ns_solver* s, Mat& D, const Mat* X, const Mat& Y, const Mat* E1, const Mat* E2,
       double diag, double scale, bool want_norm, Kind kind) {
  hipEvent_t eb = nullptr, ee = nullptr;
  if (s->timing) {
    eb = take_event(s);
    ee = take_event(s);
    if (!eb || !ee) return fail(NS_EHIP, "hipEventCreate failed");
    HIP_TRY(hipEventRecord(eb, s->stream));
  }
  int64_t np;
  int tkind;
  if (is_f64(s)) {
    GemmF64Args a{};
    a.X = X ? X->d : s->A;
    a.ldx = X ? s->ld : s->lda;
    a.Y = Y.d;
    a.ldy = s->ld;
    a.D = D.d;
    a.ldd = s->ld;
    a.E1 = E1 ? E1->d : nullptr;
    a.E2 = E2 ? E2->d : nullptr;
    a.lde1 = a.lde2 = s->ld;
    a.M = a.N = a.K = s->n;
    a.diag = diag;
    a.scale = scale;
    a.partial = want_norm ? s->partial : nullptr;
    // Only products among powers of F get a symmetric output.  The residual
    // I - A G and the G-side / merge products stay full: Newton-Schulz
    // corrects any perturbation of G only if F is the exact residual of the
    // G it multiplies, and mirroring those products would feed the part of
    // the rounding error that does not commute with A back with a gain ~kappa
    // per step.  Errors in the powers only perturb P(F) and enter F_{k+1} as
    // O(||F|| ||[A, G]||).  With S = diag(A), F = I - A S^-1 = S^(1/2) F_s
    // S^(-1/2) with F_s symmetric, so every polynomial in F has
    // D[j][i] = D[i][j] s_j / s_i: the mirror is scaled by S.
    a.sym = (s->symmetric && kind == K_POWER) ? 1 : 0;
    a.msc = (a.sym && s->diag_scale) ? s->sdiag : nullptr;
    a.sk = s->sk;
    a.sk_cap = s->sk_cap;
    np = launch_gemm_f64(a, s->stream);
    tkind = 1;
  } else {
    GemmLpArgs a{};
    const bool bf = mixed_prec(s->precision) && kind == K_POWER;
    const bool split = s->precision == NS_PREC_MIXED_SPLIT && kind != K_POWER;
    a.X = bf ? (const void*)X->b : (const void*)(X ? X->f : s->A32);
    a.Y = bf ? (const void*)Y.b : (const void*)Y.f;
    a.ldx = a.ldy = s->ld;
    if (split) {
      // X row-major (A's planes are split once per bind), Y transposed.
      const SplitPlanes& sp = s->sp;
      if (X) {
        split_operand(X->f, s->ld, s->n, s->n, false, sp.xh, sp.xl, sp.ldk, sp.part, sp.exps,
                      s->stream);
        a.X = sp.xh;
        a.Xl = sp.xl;
        a.xexp = sp.exps;
      } else {
        a.X = s->Ah;
        a.Xl = s->Al;
        a.xexp = s->aexp;
      }
      split_operand(Y.f, s->ld, s->n, s->n, true, sp.yh, sp.yl, sp.ldk,
                    sp.part + kSplitMaxParts, sp.exps + 1, s->stream);
      a.Y = sp.yh;
      a.Yl = sp.yl;
      a.yexp = sp.exps + 1;
      a.ldx = a.ldy = sp.ldk;
    }
    a.D = D.f;
    a.ldd = s->ld;
    a.Db = D.b;
    a.lddb = s->ld;
    a.E1 = E1 ? E1->f : nullptr;
    a.E2 = E2 ? E2->f : nullptr;
    a.lde1 = a.lde2 = s->ld;
    a.M = a.N = a.K = s->n;
    a.diag = (float)diag;
    a.scale = (float)scale;
    a.partial = want_norm ? s->partial : nullptr;
    if (bf) {
      np = launch_gemm_bf16_nt(a, s->stream);
    } else {
      np = split ? launch_gemm_f16s_nt(a, s->stream) : launch_gemm_f32_nn(a, s->stream);
    }
    tkind = bf ? 3 : (split ? 4 : 2);
  }
  if (np < 0) return fail(NS_EHIP, "GEMM launch failed: %s", hipGetErrorString(hipGetLastError()));
  // algorithmic flop: 2 n^3, or n^2 (n + 1) when only one triangle is formed
  const double nn = (double)s->n;
  const bool half = is_f64(s) && s->symmetric && kind == K_POWER;
  const double flop = half ? nn * nn * (nn + 1.0) : 2.0 * nn * nn * nn;
  if (s->timing) {
    HIP_TRY(hipEventRecord(ee, s->stream));
    s->timed.push_back(TimedLaunch{eb, ee, tkind, flop});
  }
  s->mmm += 1;
  s->flop += flop;
  if (want_norm) launch_reduce(s->partial, np, s->scal + 1, 2, 0.0, s->stream);
  return NS_OK;
}

int read_scalars(ns_solver* s, double* host, int first, int count) {
  HIP_TRY(hipMemcpyAsync(host, s->scal + first, count * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return NS_OK;
}

const double* sdiag_of(const ns_solver* s) { return s->diag_scale ? s->sdiag : nullptr; }

// Dst = S^-1 (I + C) (C may be null: Dst = S^-1); S = alpha I or diag(A).
void scaled_identity(ns_solver* s, const Mat* C, Mat& Dst) {
  if (is_f64(s))
    launch_scaled_identity_plus<double>(C ? C->d : nullptr, s->ld, s->n, s->scal + 0, sdiag_of(s),
                                        Dst.d, s->ld, s->stream);
  else
    launch_scaled_identity_plus<float>(C ? C->f : nullptr, s->ld, s->n, s->scal + 0, sdiag_of(s),
                                       Dst.f, s->ld, s->stream);
}

// G_next = G (I + C): GEMM, or (I + C) / alpha while G is still I / alpha.
int apply_g(ns_solver* s, const Mat& Gcur, bool implicit, const Mat& C, Mat& Gnext) {
  if (implicit) {
    scaled_identity(s, &C, Gnext);
    return NS_OK;
  }
  return mm(s, Gnext, &Gcur, C, &Gcur, nullptr, 0.0, 1.0, false, K_APPLY);
}

// C with P(Y) = I + C = (I + Y)(I + Y^2)...(I + Y^(2^(s-1))), order 2^s
// (Tables 1-2): powers into P0/P1, identity-offset assembly into C0/C1.
// Returns the matrix holding C (Y itself for order 2).
int poly_squaring(ns_solver* s, int order, const Mat& Y, const Mat** out, bool y2_ready = false) {
  int sexp = 0;
  while ((1 << sexp) < order) ++sexp;
  const Mat* pw = &Y;
  const Mat* c = &Y;
  for (int i = 1; i < sexp; ++i) {
    Mat* npw = (pw == &s->P[0]) ? &s->P[1] : &s->P[0];
    int rc = NS_OK;
    if (!(i == 1 && y2_ready))  // Y^2 may already sit in P[0]
      rc = mm(s, *npw, pw, *pw, nullptr, nullptr, 0.0, 1.0, false, K_POWER);  // Y^(2^i)
    if (rc) return rc;
    Mat* nc = (c == &s->C[0]) ? &s->C[1] : &s->C[0];
    rc = mm(s, *nc, c, *npw, c, npw, 0.0, 1.0, false, K_POWER);  // C + Y^(2^i) + C Y^(2^i)
    if (rc) return rc;
    pw = npw;
    c = nc;
  }
  *out = c;
  return NS_OK;
}

bool is_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

// C with P(Y) = I + C = I + Y + ... + Y^(order-1) for the composite loops:
// the squaring program when order = 2^s, otherwise Horner in identity-offset
// form, C <- Y + Y C (order - 2 products; eq. z1).
int poly_any(ns_solver* s, int order, const Mat& Y, const Mat** out) {
  if (is_pow2(order)) return poly_squaring(s, order, Y, out);
  const Mat* c = &Y;
  for (int j = 2; j < order; ++j) {
    Mat* nc = (c == &s->C[0]) ? &s->C[1] : &s->C[0];
    if (int rc = mm(s, *nc, &Y, *c, &Y, nullptr, 0.0, 1.0, false, K_POWER)) return rc;
    c = nc;
  }
  *out = c;
  return NS_OK;
}

int resid_into(ns_solver* s, Mat& D, const Mat& X, bool want_norm) {
  return mm(s, D, nullptr, X, nullptr, nullptr, 1.0, -1.0, want_norm, K_RESID);  // I - A X
}

// Classical step G_k = G_{k-1} P(F_{k-1}) for the non-composite forms;
// leaves G in s->G[s->gcur].
int step_classic(ns_solver* s, int order, int fact, int p, int w) {
  if (fact != NS_FACT_SQUARING) s->p0_is_f2 = false;
  Mat& Gc = s->G[s->gcur];
  Mat& Gn = s->G[s->gcur ^ 1];
  if (s->g_implicit && s->diag_scale && fact != NS_FACT_SQUARING) {
    // The Horner / unified chains add G_0 through the GEMM's scalar diagonal
    // term, which cannot hold diag(A)^-1: materialise G_0 first.
    scaled_identity(s, nullptr, Gc);
    s->g_implicit = false;
  }
  const bool impl = s->g_implicit;
  const double inv_alpha = 1.0 / s->alpha;
  int rc = NS_OK;
  if (fact == NS_FACT_SQUARING) {
    const Mat* c = nullptr;
    rc = poly_squaring(s, order, s->F, &c, s->p0_is_f2);
    s->p0_is_f2 = false;
    if (rc) return rc;
    rc = apply_g(s, Gc, impl, *c, Gn);
    if (rc) return rc;
  } else if (fact == NS_FACT_HORNER || fact == NS_FACT_UNIFIED || fact == NS_FACT_UNIFIED_PLUS1) {
    // Horner chain U_d = G + U_{d-1} F (eq. z1 / u1), d = 1..hd.
    int hd = order - 1;
    if (fact == NS_FACT_UNIFIED || fact == NS_FACT_UNIFIED_PLUS1) hd = p;
    const bool plain = (fact == NS_FACT_HORNER) || (fact == NS_FACT_UNIFIED && w == 1);
    Mat* bufs[2] = {&s->C[0], &s->C[1]};
    const Mat* u = &Gc;  // U_0 = G (may be implicit)
    bool u_impl = impl;
    for (int d = 1; d <= hd; ++d) {
      Mat* dst = (plain && d == hd) ? &Gn : bufs[d & 1];
      if (u_impl) {
        scaled_identity(s, &s->F, *dst);
      } else {
        rc = mm(s, *dst, u, s->F, impl ? nullptr : &Gc, nullptr, impl ? inv_alpha : 0.0, 1.0,
                false, K_APPLY);
        if (rc) return rc;
      }
      u = dst;
      u_impl = false;
    }
    if (!plain) {
      // Unified: Y^{p+1} = I - A U (eq. ua1), Z_i = Z_{i-1} Y^{p+1} + U (eq. zi1).
      const Mat* uu = u;
      if (u_impl) {  // p == 0 with G = I / alpha: materialise U = G
        scaled_identity(s, nullptr, s->C[0]);
        uu = &s->C[0];
      }
      const Mat* yp1 = &s->F;
      if (p > 0 && w > 1) {
        rc = resid_into(s, s->P[0], *uu, false);
        if (rc) return rc;
        yp1 = &s->P[0];
      }
      const Mat* z = uu;
      const bool plus1 = (fact == NS_FACT_UNIFIED_PLUS1);
      Mat* zb[2] = {&s->P[1], (uu == &s->C[0]) ? &s->C[1] : &s->C[0]};
      for (int i = 1; i <= w - 1; ++i) {
        Mat* dst = (!plus1 && i == w - 1) ? &Gn : zb[i & 1];
        rc = mm(s, *dst, z, *yp1, uu, nullptr, 0.0, 1.0, false, K_APPLY);
        if (rc) return rc;
        z = dst;
      }
      if (plus1) {
        // Z_1 = G + Z F (eq. ztab2).
        if (impl)
          rc = mm(s, Gn, z, s->F, nullptr, nullptr, inv_alpha, 1.0, false, K_APPLY);
        else
          rc = mm(s, Gn, z, s->F, &Gc, nullptr, 0.0, 1.0, false, K_APPLY);
        if (rc) return rc;
      }
    }
  } else {
    return fail(NS_EINVAL, "unsupported factorization %d", fact);
  }
  s->gcur ^= 1;
  s->g_implicit = false;
  return resid_into(s, s->F, s->G[s->gcur], true);  // F_k = I - A G_k
}

// D = X + Y element-wise for matrices of the solver (bf16 copy kept in mixed
// mode).
void add_into(ns_solver* s, Mat& D, const Mat& X, const Mat& Y) {
  if (is_f64(s))
    launch_add<double>(X.d, Y.d, D.d, nullptr, s->ld, s->n, s->stream);
  else
    launch_add<float>(X.f, Y.f, D.f, D.b, s->ld, s->n, s->stream);
}

// Nested programs of the tables, right orientation (Y = F_k = I - A X):
//  * order 11 (Table 2, second form): the polynomial
//    (Y + Y^2)(I + (Y^2 + Y^4)(I + Y^4)) is formed from Y^2, Y^4 first and
//    applied to X last; with the next residual, 6 products per step.
//  * order 15 (Table 3): U = X (I + Y + Y^2), Y^3 = I - A U (eq. ua1), then
//    Z = U (I + (I + Y^6)(Y^3 + Y^6)); 7 products.
//  * order 45 (eqs. ex1-ex3): U3 = X (I + Y + Y^2) (the polynomial of
//    eq. ex1 written in Y), Y^3 = I - A U3, U9 = U3 (I + Y^3 + Y^6),
//    Y^9 = I - A U9, Z = U9 (I + (I + Y^18)(Y^9 + Y^18)); 10 products.
// Every factor I + W is applied as X + X W, the powers and sums of powers are
// products among polynomials in one residual (K_POWER), and each
// intermediate residual is a full product, as in the other forms.
int step_table(ns_solver* s, int order) {
  const bool f2_ready = s->p0_is_f2;  // P[0] holds F^2 from the floor test
  s->p0_is_f2 = false;
  Mat& Gc = s->G[s->gcur];
  Mat& Gn = s->G[s->gcur ^ 1];
  const bool impl = s->g_implicit;
  Mat &F = s->F, &P0 = s->P[0], &P1 = s->P[1], &C0 = s->C[0], &C1 = s->C[1];
  int rc = NS_OK;
#define NSR_TRY(x) \
  if ((rc = (x)) != NS_OK) return rc
  if (order == 11) {
    if (!f2_ready) NSR_TRY(mm(s, P0, &F, F, nullptr, nullptr, 0.0, 1.0, false, K_POWER));  // Y^2
    NSR_TRY(mm(s, P1, &P0, P0, nullptr, nullptr, 0.0, 1.0, false, K_POWER));  // Y^4
    add_into(s, C0, P0, P1);                                                 // S = Y^2 + Y^4
    NSR_TRY(mm(s, C1, &C0, P1, &C0, nullptr, 0.0, 1.0, false, K_POWER));      // V = S + S Y^4
    add_into(s, P1, F, P0);                                                  // T = Y + Y^2
    NSR_TRY(mm(s, C0, &P1, C1, &P1, nullptr, 0.0, 1.0, false, K_POWER));      // C = T + T V
    NSR_TRY(apply_g(s, Gc, impl, C0, Gn));                                   // X (I + C)
    s->gcur ^= 1;
  } else if (order == 15 || order == 45) {
    if (f2_ready)
      add_into(s, P0, P0, F);                                                // Y + Y^2
    else
      NSR_TRY(mm(s, P0, &F, F, &F, nullptr, 0.0, 1.0, false, K_POWER));
    NSR_TRY(apply_g(s, Gc, impl, P0, Gn));                                   // U = X (I + Y + Y^2)
    NSR_TRY(resid_into(s, F, Gn, false));                                    // Y^3 = I - A U
    if (order == 15) {
      NSR_TRY(mm(s, P1, &F, F, nullptr, nullptr, 0.0, 1.0, false, K_POWER));  // Y^6
      add_into(s, C0, P1, F);                                                // S = Y^3 + Y^6
      NSR_TRY(mm(s, C1, &P1, C0, &C0, nullptr, 0.0, 1.0, false, K_POWER));    // W = S + Y^6 S
      NSR_TRY(mm(s, Gc, &Gn, C1, &Gn, nullptr, 0.0, 1.0, false, K_APPLY));    // Z = U + U W
    } else {
      NSR_TRY(mm(s, C0, &F, F, &F, nullptr, 0.0, 1.0, false, K_POWER));       // Y^3 + Y^6
      NSR_TRY(mm(s, Gc, &Gn, C0, &Gn, nullptr, 0.0, 1.0, false, K_APPLY));    // U9
      NSR_TRY(resid_into(s, F, Gc, false));                                  // Y^9 = I - A U9
      NSR_TRY(mm(s, P1, &F, F, nullptr, nullptr, 0.0, 1.0, false, K_POWER));  // Y^18
      add_into(s, C0, F, P1);                                                // S = Y^9 + Y^18
      NSR_TRY(mm(s, C1, &P1, C0, &C0, nullptr, 0.0, 1.0, false, K_POWER));    // W = S + Y^18 S
      NSR_TRY(mm(s, Gn, &Gc, C1, &Gc, nullptr, 0.0, 1.0, false, K_APPLY));    // Z = U9 + U9 W
      s->gcur ^= 1;
    }
  } else {
    return fail(NS_EINVAL, "no nested table program for order %d (11, 15, 45)", order);
  }
#undef NSR_TRY
  s->g_implicit = false;
  return resid_into(s, s->F, s->G[s->gcur], true);  // F_k = I - A G_k
}

// Precalculation of Section 5.1: T_0 = G_0, Gamma_0 = F_0,
// L_0 = T_0 P(Gamma_0), Gamma_1 = I - A L_0.
int composite_start(ns_solver* s, int order) {
  if (!s->g_implicit) return fail(NS_ESTATE, "composite form must start from G_0");
  const Mat* c = nullptr;
  int rc = poly_any(s, order, s->F, &c);
  if (rc) return rc;
  s->lcur = 0;
  scaled_identity(s, c, s->L[0]);
  rc = resid_into(s, s->Gam, s->L[0], false);
  if (rc) return rc;
  s->dns_started = true;
  return NS_OK;
}

// Double Newton-Schulz step (Section 5.1, right orientation).
int step_composite(ns_solver* s, int order) {
  int rc;
  s->p0_is_f2 = false;  // P[0] is reused by the L-loop first
  const Mat* c = nullptr;
  if (!s->dns_started) {
    if ((rc = composite_start(s, order))) return rc;
  }
  // L-loop: L_k = L_{k-1} P(Gamma_k) (lkk1), Gamma_k^n = I - A L_k (gamk21).
  rc = poly_any(s, order, s->Gam, &c);
  if (rc) return rc;
  Mat& Lc = s->L[s->lcur];
  Mat& Ln = s->L[s->lcur ^ 1];
  rc = mm(s, Ln, &Lc, *c, &Lc, nullptr, 0.0, 1.0, false, K_APPLY);
  if (rc) return rc;
  s->lcur ^= 1;
  rc = resid_into(s, s->Gam, Ln, false);
  if (rc) return rc;
  // Ordinary loop: H = G_{k-1} P(F_{k-1}).
  rc = poly_any(s, order, s->F, &c);
  if (rc) return rc;
  rc = apply_g(s, s->G[s->gcur], s->g_implicit, *c, s->H);
  if (rc) return rc;
  // Merge: G_k = L_k + H Gamma_k^n (gkgen21); F_k = I - A G_k (fks1).
  Mat& Gn = s->G[s->gcur ^ 1];
  rc = mm(s, Gn, &s->H, s->Gam, &Ln, nullptr, 0.0, 1.0, false, K_APPLY);
  if (rc) return rc;
  s->gcur ^= 1;
  s->g_implicit = false;
  return resid_into(s, s->F, Gn, true);
}

// D = X (same layout; data and bf16 copy).
int copy_mat(ns_solver* s, Mat& D, const Mat& X) {
  const size_t nn = (size_t)s->n * s->ld;
  if (is_f64(s)) {
    HIP_TRY(hipMemcpyAsync(D.d, X.d, nn * 8, hipMemcpyDeviceToDevice, s->stream));
  } else {
    HIP_TRY(hipMemcpyAsync(D.f, X.f, nn * 4, hipMemcpyDeviceToDevice, s->stream));
  }
  if (D.b && X.b) HIP_TRY(hipMemcpyAsync(D.b, X.b, nn * 2, hipMemcpyDeviceToDevice, s->stream));
  return NS_OK;
}

// Dst = G_k, materialising G_0 = S^-1 when it is still implicit.
const Mat* explicit_g(ns_solver* s) {
  if (s->g_implicit) {
    scaled_identity(s, nullptr, s->G[s->gcur]);
    s->g_implicit = false;
  }
  return &s->G[s->gcur];
}

// Remark 2 ([sri]), right orientation: Z_k = Z_{k-1} P_p(L_{k-1}),
// L_k = I - A Z_k, G_k = G_{k-1} + Z_k F_{k-1}, F_k = I - A G_k.  Z lives in
// L[0..1], L_k in Gam; Z_0 = G_0 and L_0 = F_0.
int step_sri(ns_solver* s, int order) {
  int rc;
  s->p0_is_f2 = false;
  const Mat* c = nullptr;
  if (!s->dns_started) {
    if (!s->g_implicit) return fail(NS_ESTATE, "the [sri] form must start from G_0");
    if ((rc = poly_any(s, order, s->F, &c))) return rc;
    s->lcur = 0;
    scaled_identity(s, c, s->L[0]);                                 // Z_1 = G_0 P(F_0)
    s->dns_started = true;
  } else {
    if ((rc = poly_any(s, order, s->Gam, &c))) return rc;
    Mat& Zc = s->L[s->lcur];
    Mat& Zn = s->L[s->lcur ^ 1];
    if ((rc = mm(s, Zn, &Zc, *c, &Zc, nullptr, 0.0, 1.0, false, K_APPLY))) return rc;
    s->lcur ^= 1;
  }
  Mat& Z = s->L[s->lcur];
  if ((rc = resid_into(s, s->Gam, Z, false))) return rc;            // L_k = I - A Z_k
  const Mat* Gc = explicit_g(s);
  Mat& Gn = s->G[s->gcur ^ 1];
  if ((rc = mm(s, Gn, &Z, s->F, Gc, nullptr, 0.0, 1.0, false, K_APPLY))) return rc;
  s->gcur ^= 1;
  return resid_into(s, s->F, Gn, true);
}

// General composite expansion (eqs. gkgen1-ga1), right orientation, with
// s->gc_w loops of orders m_i: loop i holds T_i = S^-1 sum_{j < x_i}
// (S^-1 D)^j and Gamma_i = I - A T_i with x_i = m_i^(k-1) before step k.
//   T_i <- T_i P_{m_i}(Gamma_i),  Gamma_i <- I - A T_i
//   T_c = T_1 + (T_2 + T_3 Gamma_2) Gamma_1,  Gamma_c = Gamma_3 Gamma_2 Gamma_1
//   G_k = T_c + G_{k-1} P_n(F_{k-1}) Gamma_c,   F_k = I - A G_k = F_{k-1}^n Gamma_c
int step_gc(ns_solver* s, int order) {
  int rc;
  s->p0_is_f2 = false;
  const int w = s->gc_w;
  const Mat* c = nullptr;
  if (!s->gc_started) {
    if (!s->g_implicit) return fail(NS_ESTATE, "the composite form must start from G_0");
    for (int i = 0; i < w; ++i) {
      s->tcur[i] = 0;
      if (s->gc_m[i] == 1) {   // x_i = 1 for ever: T_i = S^-1, Gamma_i = F_0
        scaled_identity(s, nullptr, *s->loopT[i][0]);
        if ((rc = copy_mat(s, *s->loopG[i], s->F))) return rc;
      }
    }
  }
  // 1. loops (Gamma_i of a fresh loop is F_0 = s->F)
  for (int i = 0; i < w; ++i) {
    const int m = s->gc_m[i];
    if (m == 1) continue;
    if (!s->gc_started) {
      if ((rc = poly_any(s, m, s->F, &c))) return rc;
      scaled_identity(s, c, *s->loopT[i][0]);
    } else {
      if ((rc = poly_any(s, m, *s->loopG[i], &c))) return rc;
      Mat& Tc = *s->loopT[i][s->tcur[i]];
      Mat& Tn = *s->loopT[i][s->tcur[i] ^ 1];
      if ((rc = mm(s, Tn, &Tc, *c, &Tc, nullptr, 0.0, 1.0, false, K_APPLY))) return rc;
      s->tcur[i] ^= 1;
    }
    if ((rc = resid_into(s, *s->loopG[i], *s->loopT[i][s->tcur[i]], false))) return rc;
  }
  // 2. ordinary loop H = G_{k-1} P_n(F_{k-1})
  const Mat* H;
  if (order >= 2) {
    if ((rc = poly_any(s, order, s->F, &c))) return rc;
    if ((rc = apply_g(s, s->G[s->gcur], s->g_implicit, *c, s->H))) return rc;
    H = &s->H;
  } else {
    H = explicit_g(s);
  }
  // 3. composite polynomial and residual
  const Mat* T1 = s->loopT[0][s->tcur[0]];
  const Mat* tc = T1;
  const Mat* gcm = s->loopG[0];
  if (w >= 2) {
    const Mat* T2 = s->loopT[1][s->tcur[1]];
    const Mat* inner = T2;
    if (w == 3) {   // T_2 + T_3 Gamma_2
      if ((rc = mm(s, s->C[0], s->loopT[2][s->tcur[2]], *s->loopG[1], T2, nullptr, 0.0, 1.0,
                   false, K_APPLY)))
        return rc;
      inner = &s->C[0];
    }
    if ((rc = mm(s, s->P[0], inner, *s->loopG[0], T1, nullptr, 0.0, 1.0, false, K_APPLY)))
      return rc;
    tc = &s->P[0];
    const Mat* g21 = s->loopG[1];
    if (w == 3) {   // Gamma_3 Gamma_2
      if ((rc = mm(s, s->C[1], s->loopG[2], *s->loopG[1], nullptr, nullptr, 0.0, 1.0, false,
                   K_POWER)))
        return rc;
      g21 = &s->C[1];
    }
    if ((rc = mm(s, s->P[1], g21, *s->loopG[0], nullptr, nullptr, 0.0, 1.0, false, K_POWER)))
      return rc;
    gcm = &s->P[1];
  }
  // 4. merge and residual
  Mat& Gn = s->G[s->gcur ^ 1];
  if ((rc = mm(s, Gn, H, *gcm, tc, nullptr, 0.0, 1.0, false, K_APPLY))) return rc;
  s->gcur ^= 1;
  s->g_implicit = false;
  s->gc_started = true;
  return resid_into(s, s->F, Gn, true);
}

// y = M x + z (accumulate: y += M x + z) for an iterate M of the solver.
void mat_vec(ns_solver* s, const Mat& M, const double* x, const double* z, double* y,
             int accumulate) {
  if (is_f64(s))
    launch_gemv<double>(M.d, s->ld, s->n, x, z, y, accumulate, s->stream);
  else
    launch_gemv<float>(M.f, s->ld, s->n, x, z, y, accumulate, s->stream);
}

// theta += omega_k r with the accelerator of eq. (ttk1), right orientation:
// omega r = L_k r + G_k {sum_{j<q} F_k^j} Gamma_k^n r (r = s->r).
void accel_apply(ns_solver* s, int q, double* theta) {
  mat_vec(s, s->Gam, s->r, nullptr, s->vt, 0);                 // t = Gamma^n r
  const double* w = s->vt;
  for (int j = 1; j < q; ++j) {                                // w = t + F w (Horner)
    double* nw = s->vw[j & 1];
    mat_vec(s, s->F, w, s->vt, nw, 0);
    w = nw;
  }
  double* v = (w == s->vw[0]) ? s->vw[1] : s->vw[0];
  mat_vec(s, s->G[s->gcur], w, nullptr, v, 0);                 // v = G w
  mat_vec(s, s->L[s->lcur], s->r, v, theta, 1);                // theta += L r + v
}

void gemv_update(ns_solver* s, double* theta) {
  const Mat& G = s->G[s->gcur];
  if (is_f64(s))
    launch_gemv_update<double>(G.d, s->ld, s->n, s->r, theta, s->stream);
  else
    launch_gemv_update<float>(G.f, s->ld, s->n, s->r, theta, s->stream);
}

int any_step(ns_solver* s, int order, int fact, int p, int w) {
  switch (fact) {
    case NS_FACT_COMPOSITE_DOUBLE: return step_composite(s, order);
    case NS_FACT_TABLE: return step_table(s, order);
    case NS_FACT_SRI: return step_sri(s, order);
    case NS_FACT_COMPOSITE_GENERAL: return step_gc(s, order);
    default: return step_classic(s, order, fact, p, w);
  }
}

int check_solver(ns_solver* s) {
  if (!s) return fail(NS_EINVAL, "null solver");
  return NS_OK;
}

int richardson_once(ns_solver* s, const double* b, double* theta) {
  const int64_t np = launch_gemv_resid(s->A, s->lda, s->n, b, theta, s->r, s->partial, s->stream);
  launch_reduce(s->partial, np, s->scal + 2, 2, 0.0, s->stream);
  if (s->g_implicit) {
    launch_vec_scale(s->r, s->scal + 0, sdiag_of(s), theta, s->n, 1, s->stream);
  } else {
    gemv_update(s, theta);
  }
  return NS_OK;
}

// The fixed-length Newton-Schulz phase: k_max steps, each followed by the
// Richardson update with the new G and a device-side record of ||F_k|| and
// ||r||.  No host decision depends on a device value, so the sequence is
// captured once into a HIP graph (per operands and options) and replayed; the
// host-side state the steps leave behind is saved with it.
int enqueue_fixed(ns_solver* s, const ns_solve_opts* o, const double* b, double* theta) {
  for (int k = 1; k <= o->k_max; ++k) {
    if (int rc = any_step(s, o->order, o->factorization, o->p, o->w)) return rc;
    richardson_once(s, b, theta);
    launch_record(s->scal, s->dhist, s->dhist + NS_HIST_F, k, s->stream);
  }
  return NS_OK;
}

int run_fixed_graph(ns_solver* s, const ns_solve_opts* o, const double* b, double* theta) {
  ns_solver::GraphKey key{o->order, o->factorization, o->p, o->w, o->k_max, s->precision,
                          s->symmetric ? 1 : 0, s->diag_scale ? 1 : 0, s->A, b, theta, s->lda};
  if (!s->graph_exec || !(key == s->graph_key)) {
    if (s->graph_exec) {
      (void)hipGraphExecDestroy(s->graph_exec);
      s->graph_exec = nullptr;
    }
    const int64_t mmm0 = s->mmm;
    const double flop0 = s->flop;
    // Capture on a private stream (the caller's may be the null stream, which
    // cannot be captured); the graph is launched on the caller's stream.
    if (!s->capture_stream)
      HIP_TRY(hipStreamCreateWithFlags(&s->capture_stream, hipStreamNonBlocking));
    hipStream_t user = s->stream;
    s->stream = s->capture_stream;
    hipError_t eb = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
      s->stream = user;
      return fail(NS_EHIP, "hipStreamBeginCapture failed: %s", hipGetErrorString(eb));
    }
    int rc = enqueue_fixed(s, o, b, theta);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s->stream, &g);
    s->stream = user;
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess || !g) return fail(NS_EHIP, "graph capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      s->graph_exec = nullptr;
      return fail(NS_EHIP, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    s->graph_key = key;
    s->graph_gcur = s->gcur;
    s->graph_mmm = s->mmm - mmm0;
    s->graph_flop = s->flop - flop0;
  } else {
    // Replay: put the host-side state where the captured steps leave it.
    s->gcur = s->graph_gcur;
    s->g_implicit = false;
    s->p0_is_f2 = false;
    s->mmm += s->graph_mmm;
    s->flop += s->graph_flop;
  }
  HIP_TRY(hipGraphLaunch(s->graph_exec, s->stream));
  return NS_OK;
}

int validate_step_args(ns_solver* s, int order, int fact, int p, int w) {
  if (order < (fact == NS_FACT_COMPOSITE_GENERAL ? 1 : 2))
    return fail(NS_EINVAL, "order must be >= 2 (got %d)", order);
  switch (fact) {
    case NS_FACT_HORNER:
      return NS_OK;
    case NS_FACT_SQUARING:
      if (!is_pow2(order)) return fail(NS_EINVAL, "squaring form needs order = 2^s (got %d)", order);
      return NS_OK;
    case NS_FACT_UNIFIED:
      if (p < 0 || w < 1 || w * (p + 1) != order)
        return fail(NS_EINVAL, "unified form needs order = w (p + 1)");
      return NS_OK;
    case NS_FACT_UNIFIED_PLUS1:
      if (p < 0 || w < 1 || w * (p + 1) + 1 != order)
        return fail(NS_EINVAL, "unified+1 form needs order = w (p + 1) + 1");
      return NS_OK;
    case NS_FACT_TABLE:
      if (order != 11 && order != 15 && order != 45)
        return fail(NS_EINVAL, "table programs exist for orders 11, 15, 45 (got %d)", order);
      return NS_OK;
    case NS_FACT_SRI:
      if (!s->composite_capable)
        return fail(NS_EINVAL, "workspace was sized without the composite buffers");
      return NS_OK;
    case NS_FACT_COMPOSITE_GENERAL:
      if (s->gc_w < 1) return fail(NS_ESTATE, "ns_set_composite_rates first");
      if (s->composite_capable < s->gc_w)
        return fail(NS_EINVAL, "workspace was sized for fewer composite loops");
      return NS_OK;
    case NS_FACT_COMPOSITE_DOUBLE:
      if (!s->composite_capable)
        return fail(NS_EINVAL, "workspace was sized without the composite buffers");
      return NS_OK;
    default:
      return fail(NS_EINVAL, "unknown factorization %d", fact);
  }
}

}  // namespace

extern "C" {

const char* ns_version(void) { return "nsr 0.1 (gfx950)"; }

const char* ns_last_error(void) { return g_err; }

const char* ns_status_string(int st) {
  switch (st) {
    case NS_OK: return "ok";
    case NS_EINVAL: return "invalid argument";
    case NS_ENOTSPD: return "matrix is not SPD (alpha not positive/finite)";
    case NS_EDIVERGED: return "iteration diverged";
    case NS_ENOCONV: return "tolerance not reached";
    case NS_ENOMEM: return "workspace too small";
    case NS_EHIP: return "HIP runtime error";
    case NS_EBUSY: return "not finished";
    case NS_EPRECISION: return "precision insufficient";
    case NS_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

size_t ns_workspace_bytes(int64_t n, int precision, int composite) {
  if (n < 1) return 0;
  if (precision < NS_PREC_FP64 || precision > NS_PREC_MIXED_SPLIT) return 0;
  if (composite < 0 || composite > kMaxLoops) return 0;
  return layout_bytes(n, precision, composite);
}

int ns_create(int device, void* hip_stream, int64_t n, int precision, void* workspace,
              size_t bytes, ns_solver** out) {
  if (!out) return fail(NS_EINVAL, "null out");
  *out = nullptr;
  if (n < 1) return fail(NS_EINVAL, "n must be >= 1");
  if (n > 65535) return fail(NS_EINVAL, "n must be <= 65535");
  if (precision < NS_PREC_FP64 || precision > NS_PREC_MIXED_SPLIT)
    return fail(NS_EINVAL, "unknown precision %d", precision);
  if (!workspace) return fail(NS_EINVAL, "null workspace");
  if ((reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return fail(NS_EINVAL, "workspace must be 256-byte aligned");
  const size_t need_plain = layout_bytes(n, precision, 0);
  if (bytes < need_plain)
    return fail(NS_ENOMEM, "workspace too small: %zu < %zu bytes", bytes, need_plain);
  HIP_TRY(hipSetDevice(device));
  ns_solver* s = new (std::nothrow) ns_solver();
  if (!s) return fail(NS_ENOMEM, "host allocation failed");
  s->device = device;
  s->stream = reinterpret_cast<hipStream_t>(hip_stream);
  s->n = n;
  s->ld = ld_for(n);
  s->precision = precision;
  s->composite_capable = 0;
  for (int lv = 1; lv <= kMaxLoops; ++lv)
    if (bytes >= layout_bytes(n, precision, lv)) s->composite_capable = lv;
  s->ws = reinterpret_cast<char*>(workspace);
  s->ws_bytes = bytes;
  const size_t nn = (size_t)n * s->ld;
  const size_t mat = align_up(nn * elem_bytes(precision), kAlign);
  const size_t shadow = align_up(nn * 2, kAlign);
  char* p = s->ws;
  auto take = [&](size_t b) {
    char* q = p;
    p += b;
    return q;
  };
  auto mat_of = [&](Mat& m, bool with_shadow) {
    char* q = take(mat);
    if (precision == NS_PREC_FP64)
      m.d = reinterpret_cast<double*>(q);
    else
      m.f = reinterpret_cast<float*>(q);
    if (with_shadow && mixed_prec(precision)) m.b = reinterpret_cast<uint16_t*>(take(shadow));
  };
  mat_of(s->G[0], false);
  mat_of(s->G[1], false);
  mat_of(s->F, true);
  mat_of(s->P[0], true);
  mat_of(s->P[1], true);
  mat_of(s->C[0], true);
  mat_of(s->C[1], true);
  if (s->composite_capable >= 1) {
    mat_of(s->L[0], false);
    mat_of(s->L[1], false);
    mat_of(s->Gam, true);
    mat_of(s->H, false);
    s->loopT[0][0] = &s->L[0];
    s->loopT[0][1] = &s->L[1];
    s->loopG[0] = &s->Gam;
  }
  for (int i = 1; i < s->composite_capable; ++i) {
    mat_of(s->LT[i - 1][0], false);
    mat_of(s->LT[i - 1][1], false);
    mat_of(s->LG[i - 1], true);
    s->loopT[i][0] = &s->LT[i - 1][0];
    s->loopT[i][1] = &s->LT[i - 1][1];
    s->loopG[i] = &s->LG[i - 1];
  }
  if (precision != NS_PREC_FP64) s->A32 = reinterpret_cast<float*>(take(align_up(nn * 4, kAlign)));
  if (precision == NS_PREC_MIXED_SPLIT) {
    const size_t plane = align_up((size_t)n * split_ld(n) * 2, kAlign);
    s->Ah = reinterpret_cast<uint16_t*>(take(plane));
    s->Al = reinterpret_cast<uint16_t*>(take(plane));
    s->aexp = reinterpret_cast<float*>(take(align_up(sizeof(float), kAlign)));
    s->sp = carve_split(take(split_scratch_bytes(n, n, n)), n, n, n);
  }

  s->r = reinterpret_cast<double*>(take(align_up((size_t)n * sizeof(double), kAlign)));
  s->vt = reinterpret_cast<double*>(take(align_up((size_t)n * sizeof(double), kAlign)));
  s->vw[0] = reinterpret_cast<double*>(take(align_up((size_t)n * sizeof(double), kAlign)));
  s->vw[1] = reinterpret_cast<double*>(take(align_up((size_t)n * sizeof(double), kAlign)));
  s->sdiag = reinterpret_cast<double*>(take(align_up((size_t)n * sizeof(double), kAlign)));
  s->partial =
      reinterpret_cast<double*>(take(align_up((size_t)partial_capacity(n) * sizeof(double), kAlign)));
  s->scal = reinterpret_cast<double*>(take(align_up(16 * sizeof(double), kAlign)));
  s->dhist = reinterpret_cast<double*>(
      take(align_up((NS_HIST_F + NS_HIST_R) * sizeof(double), kAlign)));
  if (precision == NS_PREC_FP64) {
    const size_t skb = split_bytes(n);
    if (skb > 0) {
      s->sk = reinterpret_cast<double*>(take(align_up(skb, kAlign)));
      s->sk_cap = (int64_t)(skb / sizeof(double));
    }
  }
  if ((size_t)(p - s->ws) > bytes) {  // layout_bytes and this carving must agree
    delete s;
    return fail(NS_ENOMEM, "internal layout exceeds workspace");
  }
  *out = s;
  return NS_OK;
}

int ns_destroy(ns_solver* s) {
  if (!s) return NS_OK;
  if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
  if (s->capture_stream) (void)hipStreamDestroy(s->capture_stream);
  for (hipEvent_t e : s->pool) (void)hipEventDestroy(e);
  delete s;
  return NS_OK;
}

int ns_bind(ns_solver* s, const double* A, int64_t lda) {
  if (int rc = check_solver(s)) return rc;
  if (!A) return fail(NS_EINVAL, "null A");
  if (lda < s->n) return fail(NS_EINVAL, "lda < n");
  s->A = A;
  s->lda = lda;
  s->bound = true;
  s->scaled = false;
  s->g_implicit = true;
  s->dns_started = false;
  s->p0_is_f2 = false;
  s->gcur = 0;
  s->lcur = 0;
  if (!is_f64(s)) {
    HIP_TRY(hipSetDevice(s->device));
    launch_convert<double, float>(A, lda, s->n, s->A32, s->ld, s->stream);
    if (s->precision == NS_PREC_MIXED_SPLIT)
      split_operand(s->A32, s->ld, s->n, s->n, false, s->Ah, s->Al, s->sp.ldk, s->sp.part,
                    s->aexp, s->stream);
    if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  }
  return NS_OK;
}

int ns_init_scale(ns_solver* s, int scale, double eps, double* alpha_out, double* fnorm0_out) {
  if (int rc = check_solver(s)) return rc;
  if (!s->bound) return fail(NS_ESTATE, "ns_bind first");
  HIP_TRY(hipSetDevice(s->device));
  s->diag_scale = false;
  if (scale == NS_SCALE_FROBENIUS) {
    const int64_t np = launch_sumsq(s->A, s->lda, s->n, s->partial, s->stream);
    launch_reduce(s->partial, np, s->scal + 0, 2, 0.0, s->stream);
  } else if (scale == NS_SCALE_INF_HALF) {
    launch_rowabs(s->A, s->lda, s->n, s->partial, s->stream);
    launch_reduce(s->partial, s->n, s->scal + 0, 3, eps, s->stream);
  } else if (scale == NS_SCALE_DIAG) {
    if (mixed_prec(s->precision))
      return fail(NS_EINVAL, "NS_SCALE_DIAG needs the float64 or float32 mode");
    launch_diag(s->A, s->lda, s->n, s->sdiag, s->partial, s->stream);
    launch_reduce(s->sdiag, s->n, s->scal + 0, 1, 0.0, s->stream);     // max A_ii
    launch_reduce(s->partial, s->n, s->scal + 4, 1, 0.0, s->stream);   // -min A_ii
    double h2[5];
    if (int rc = read_scalars(s, h2, 0, 5)) return rc;
    if (!(-h2[4] > 0.0) || !isfinite(h2[0]) || !isfinite(h2[4]))
      return fail(NS_ENOTSPD, "diagonal entry %g is not a positive finite number", -h2[4]);
    s->diag_scale = true;
  } else {
    return fail(NS_EINVAL, "unknown scale %d", scale);
  }
  double host[1];
  if (int rc = read_scalars(s, host, 0, 1)) return rc;
  s->alpha = host[0];
  if (!(s->alpha > 0.0) || !isfinite(s->alpha))
    return fail(NS_ENOTSPD, "alpha = %g is not a positive finite number", s->alpha);
  int64_t np;
  if (is_f64(s))
    np = launch_init_resid<double>(s->A, s->lda, s->n, s->scal + 0, sdiag_of(s), s->F.d, s->ld,
                                   nullptr, s->partial, s->stream);
  else
    np = launch_init_resid<float>(s->A, s->lda, s->n, s->scal + 0, sdiag_of(s), s->F.f, s->ld,
                                  s->F.b, s->partial, s->stream);
  launch_reduce(s->partial, np, s->scal + 1, 2, 0.0, s->stream);
  s->scaled = true;
  s->g_implicit = true;
  s->dns_started = false;
  s->gc_started = false;
  s->p0_is_f2 = false;
  s->gcur = 0;
  s->lcur = 0;
  s->mmm = 0;
  s->flop = 0.0;
  if (alpha_out) *alpha_out = s->alpha;
  if (fnorm0_out) {
    if (int rc = read_scalars(s, host, 1, 1)) return rc;
    *fnorm0_out = host[0];
  }
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  return NS_OK;
}

int ns_step(ns_solver* s, int order, int factorization, int p, int w, double* fnorm_out) {
  if (int rc = check_solver(s)) return rc;
  if (!s->scaled) return fail(NS_ESTATE, "ns_init_scale first");
  if (int rc = validate_step_args(s, order, factorization, p, w)) return rc;
  HIP_TRY(hipSetDevice(s->device));
  int rc = any_step(s, order, factorization, p, w);
  if (rc) return rc;
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  if (fnorm_out) {
    double host[1];
    if ((rc = read_scalars(s, host, 1, 1))) return rc;
    *fnorm_out = host[0];
  }
  return NS_OK;
}

static int copy_out(ns_solver* s, const Mat& m, double* out, int64_t ldo) {
  if (is_f64(s)) {
    HIP_TRY(hipMemcpy2DAsync(out, ldo * sizeof(double), m.d, s->ld * sizeof(double),
                             s->n * sizeof(double), s->n, hipMemcpyDeviceToDevice, s->stream));
  } else {
    launch_convert<float, double>(m.f, s->ld, s->n, out, ldo, s->stream);
    if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  }
  return NS_OK;
}

int ns_get_G(ns_solver* s, double* G_out, int64_t ldg) {
  if (int rc = check_solver(s)) return rc;
  if (!G_out || ldg < s->n) return fail(NS_EINVAL, "bad G_out / ldg");
  if (!s->scaled) return fail(NS_ESTATE, "ns_init_scale first");
  if (s->g_implicit) {
    launch_scaled_identity_plus<double>(nullptr, 0, s->n, s->scal + 0, sdiag_of(s), G_out, ldg,
                                        s->stream);
    return NS_OK;
  }
  return copy_out(s, s->G[s->gcur], G_out, ldg);
}

int ns_get_F(ns_solver* s, double* F_out, int64_t ldf) {
  if (int rc = check_solver(s)) return rc;
  if (!F_out || ldf < s->n) return fail(NS_EINVAL, "bad F_out / ldf");
  if (!s->scaled) return fail(NS_ESTATE, "ns_init_scale first");
  return copy_out(s, s->F, F_out, ldf);
}

int ns_richardson_step(ns_solver* s, const double* b, double* theta, double* rnorm_out) {
  if (int rc = check_solver(s)) return rc;
  if (!b || !theta) return fail(NS_EINVAL, "null b / theta");
  if (!s->scaled) return fail(NS_ESTATE, "ns_init_scale first");
  richardson_once(s, b, theta);
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  if (rnorm_out) {
    double host[1];
    if (int rc = read_scalars(s, host, 2, 1)) return rc;
    *rnorm_out = host[0];
  }
  return NS_OK;
}

int richardson_ns_solve(ns_solver* s, const double* b, double* theta, const ns_solve_opts* o,
                        ns_solve_report* rep) {
  if (int rc = check_solver(s)) return rc;
  if (!b || !theta || !o) return fail(NS_EINVAL, "null b / theta / opts");
  if (o->k_max < 1 || o->k_max > NS_HIST_F - 1) return fail(NS_EINVAL, "k_max must be in 1..64");
  if (o->refine_max < 0) return fail(NS_EINVAL, "refine_max < 0");
  if (o->theta0_mode < 0 || o->theta0_mode > 2) return fail(NS_EINVAL, "bad theta0_mode");
  if (o->accel_q < 0) return fail(NS_EINVAL, "accel_q < 0");
  if (o->accel_q > 0 && o->factorization != NS_FACT_COMPOSITE_DOUBLE)
    return fail(NS_EINVAL, "the accelerator (accel_q > 0) needs the composite form");
  if (int rc = validate_step_args(s, o->order, o->factorization, o->p, o->w)) return rc;
  const int h = o->init_order > 1 ? o->init_order : 1;
  int hp = o->init_p, hw = o->init_w;
  if (o->init_order < 0 || hp < 0 || hw < 0) return fail(NS_EINVAL, "negative initial series");
  if (h > 1) {
    if (o->factorization == NS_FACT_COMPOSITE_DOUBLE || o->accel_q > 0)
      return fail(NS_EINVAL, "the initial series (init_order > 1) is for the classical forms");
    if (hp == 0 && hw == 0) {
      hp = h - 1;
      hw = 1;
    }
    if (int rc = validate_step_args(s, h, NS_FACT_UNIFIED, hp, hw)) return rc;
  }
  ns_solve_report local;
  ns_solve_report* R = rep ? rep : &local;
  memset(R, 0, sizeof(*R));
  R->precision = s->precision;

  double alpha = 0.0, f0 = 0.0;
  if (int rc = ns_init_scale(s, o->scale, o->eps, &alpha, &f0)) return rc;
  R->alpha = alpha;
  if (h > 1) {
    // G_0 = S^-1 sum_{j<h} (I - A S^-1)^j by the unified program (eq. g01),
    // F_0 = (I - A S^-1)^h (eq. g03).
    if (int rc = step_classic(s, h, NS_FACT_UNIFIED, hp, hw)) return rc;
    double hf[1];
    if (int rc = read_scalars(s, hf, 1, 1)) return rc;
    f0 = hf[0];
  }
  R->fnorm_hist[R->n_fnorm++] = f0;

  // ||b||
  {
    const int64_t np = launch_vec_sumsq(b, s->n, s->partial, s->stream);
    launch_reduce(s->partial, np, s->scal + 3, 2, 0.0, s->stream);
  }
  const int q = o->accel_q;
  if (q > 0) {
    // theta_0 = L_0 b (the accelerated scheme's start, below eq. riem6)
    if (int rc = composite_start(s, o->order)) return rc;
    mat_vec(s, s->L[s->lcur], b, nullptr, theta, 0);
  } else if (o->theta0_mode == 0) {
    if (s->g_implicit)
      launch_vec_scale(b, s->scal + 0, sdiag_of(s), theta, s->n, 0, s->stream);
    else
      mat_vec(s, s->G[s->gcur], b, nullptr, theta, 0);   // theta_0 = G_0 b
  } else if (o->theta0_mode == 1) {
    HIP_TRY(hipMemsetAsync(theta, 0, s->n * sizeof(double), s->stream));
  }
  double bn[1];
  if (int rc = read_scalars(s, bn, 3, 1)) return rc;
  double bnorm = bn[0] > 0.0 ? bn[0] : 1.0;

  int ns_stop = NS_STOP_NONE;
  if (!isfinite(f0)) ns_stop = NS_STOP_DIVERGED;
  int k = 0;
  double host[2];
  const bool fixed_len = o->graph && !o->floor_detect && !(o->f_tol > 0.0) && q == 0 &&
                         h == 1 && !s->timing &&
                         (o->factorization == NS_FACT_HORNER ||
                          o->factorization == NS_FACT_SQUARING ||
                          o->factorization == NS_FACT_TABLE ||
                          o->factorization == NS_FACT_UNIFIED ||
                          o->factorization == NS_FACT_UNIFIED_PLUS1);
  if (fixed_len && ns_stop == NS_STOP_NONE) {
    if (int rc = run_fixed_graph(s, o, b, theta)) return rc;
    k = o->k_max;
    std::vector<double> hh(NS_HIST_F + NS_HIST_R);
    HIP_TRY(hipMemcpyAsync(hh.data(), s->dhist, hh.size() * sizeof(double),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int j = 1; j <= k; ++j) {
      R->fnorm_hist[R->n_fnorm++] = hh[j];
      if (R->n_resid < NS_HIST_R) R->resid_hist[R->n_resid++] = hh[NS_HIST_F + j - 1] / bnorm;
    }
    ns_stop = NS_STOP_K_MAX;
    for (int j = 1; j <= k; ++j)
      if (!isfinite(hh[j]) || hh[j] > f0) ns_stop = NS_STOP_DIVERGED;
  }
  // Order n of the error law: F_k = F_{k-1}^n for the classical programs,
  // F_k = F_0^(k n^(k+1) + n^k) for the double Newton-Schulz (Section 5.1),
  // an exponent at least n times the previous one; so ||F_k|| <=
  // ||F_{k-1}||^n in exact arithmetic.  0: the general composite and [sri],
  // whose stop rule is the ratio test alone.
  const int law = (o->factorization == NS_FACT_HORNER || o->factorization == NS_FACT_SQUARING ||
                   o->factorization == NS_FACT_TABLE || o->factorization == NS_FACT_UNIFIED ||
                   o->factorization == NS_FACT_UNIFIED_PLUS1 ||
                   o->factorization == NS_FACT_COMPOSITE_DOUBLE)
                      ? o->order
                      : 0;
  while (ns_stop == NS_STOP_NONE) {
    ++k;
    int rc = any_step(s, o->order, o->factorization, o->p, o->w);
    if (rc) return rc;
    if (q > 0) {
      const int64_t np = launch_gemv_resid(s->A, s->lda, s->n, b, theta, s->r, s->partial, s->stream);
      launch_reduce(s->partial, np, s->scal + 2, 2, 0.0, s->stream);
      accel_apply(s, q, theta);
    } else {
      richardson_once(s, b, theta);
    }
    if ((rc = read_scalars(s, host, 1, 2))) return rc;
    const double fk = host[0];
    if (R->n_resid < NS_HIST_R) R->resid_hist[R->n_resid++] = host[1] / bnorm;
    R->fnorm_hist[R->n_fnorm++] = fk;
    // Stop rule (the paper gives none): divergence, tolerance, rounding
    // floor, k_max.  Floor: ||F_k|| > ||F_{k-1}|| / 2 although
    // ||F_k^2|| <= ||F_k|| / 4; in exact arithmetic (F_k = F_{k-1}^n, log of
    // the power sums convex in the exponent) the second forces the ratio
    // below 1/2, so rounding dominates.  F_k^2 lands in P[0], where the next
    // squaring step picks it up.
    const double* h = R->fnorm_hist;
    if (!isfinite(fk) || fk > h[0]) {
      ns_stop = NS_STOP_DIVERGED;
    } else if (fk <= o->f_tol) {
      ns_stop = NS_STOP_F_TOL;
    } else if (o->floor_detect && law > 0 && h[k - 1] < 1.0 &&
               fk > kLawMargin * pow(h[k - 1], (double)law)) {
      // Error law (eq. fk1): F_k = F_{k-1}^n gives ||F_k||_F <= ||F_{k-1}||_F^n
      // in exact arithmetic; a norm far above that is rounding error, which
      // another step reproduces, so the floor is found on the step that
      // reaches it.
      ns_stop = NS_STOP_FLOOR;
    } else {
      if (o->floor_detect && fk > 0.5 * h[k - 1]) {
        if ((rc = mm(s, s->P[0], &s->F, s->F, nullptr, nullptr, 0.0, 1.0, true, K_POWER)))
          return rc;
        if ((rc = read_scalars(s, host, 1, 1))) return rc;
        s->p0_is_f2 = true;
        if (host[0] <= 0.25 * fk) ns_stop = NS_STOP_FLOOR;
      }
      if (ns_stop == NS_STOP_NONE && k >= o->k_max) ns_stop = NS_STOP_K_MAX;
    }
  }
  R->ns_steps = k;
  R->ns_stop = ns_stop;

  int status = NS_OK;
  int refine = 0;
  double rel = NAN;
  int refine_stop = NS_STOP_DIVERGED;
  if (ns_stop != NS_STOP_DIVERGED) {
    const int hist0 = R->n_resid;
    double last[4] = {0, 0, 0, 0};
    int nlast = 0;
    while (true) {
      // r = b - A theta, ||r||; the update is applied only if we continue.
      const int64_t np =
          launch_gemv_resid(s->A, s->lda, s->n, b, theta, s->r, s->partial, s->stream);
      launch_reduce(s->partial, np, s->scal + 2, 2, 0.0, s->stream);
      if (int rc = read_scalars(s, host, 2, 1)) return rc;
      rel = host[0] / bnorm;
      if (R->n_resid < NS_HIST_R) R->resid_hist[R->n_resid++] = rel;
      for (int j = 3; j > 0; --j) last[j] = last[j - 1];
      last[0] = rel;
      ++nlast;
      if (!isfinite(rel)) {
        refine_stop = NS_STOP_DIVERGED;
        break;
      }
      if (rel <= o->resid_tol) {
        refine_stop = NS_STOP_RESID_TOL;
        break;
      }
      if (refine >= o->refine_max) {
        refine_stop = NS_STOP_REFINE_MAX;
        break;
      }
      if (refine >= 3 && nlast >= 4 && rel > 0.5 * last[3]) {
        refine_stop = NS_STOP_REFINE_STALL;
        break;
      }
      if (q > 0)
        accel_apply(s, q, theta);
      else if (s->g_implicit)
        launch_vec_scale(s->r, s->scal + 0, sdiag_of(s), theta, s->n, 1, s->stream);
      else
        gemv_update(s, theta);
      ++refine;
    }
    (void)hist0;
  }
  R->refine_steps = refine;
  R->refine_stop = refine_stop;
  R->rel_resid = rel;
  R->mmm = s->mmm;
  R->gemm_flop = s->flop;
  if (ns_stop == NS_STOP_DIVERGED || refine_stop == NS_STOP_DIVERGED)
    status = NS_EDIVERGED;
  else if (refine_stop != NS_STOP_RESID_TOL)
    status = NS_ENOCONV;
  R->status = status;
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  if (status == NS_EDIVERGED) return fail(NS_EDIVERGED, "iteration diverged");
  if (status == NS_ENOCONV) return fail(NS_ENOCONV, "resid_tol not reached (%g)", rel);
  return NS_OK;
}

int ns_set_composite_rates(ns_solver* s, int w, const int* rates) {
  if (int rc = check_solver(s)) return rc;
  if (w < 1 || w > kMaxLoops) return fail(NS_EINVAL, "w must be in 1..%d", kMaxLoops);
  if (!rates) return fail(NS_EINVAL, "null rates");
  if (w > s->composite_capable)
    return fail(NS_EINVAL, "workspace was sized for %d composite loops", s->composite_capable);
  if (s->gc_started) return fail(NS_ESTATE, "rates are set before the first composite step");
  for (int i = 0; i < w; ++i)
    if (rates[i] < 1 || rates[i] > 64)
      return fail(NS_EINVAL, "loop orders must be in 1..64 (got %d)", rates[i]);
  s->gc_w = w;
  for (int i = 0; i < kMaxLoops; ++i) s->gc_m[i] = i < w ? rates[i] : 0;
  return NS_OK;
}

int ns_set_symmetric(ns_solver* s, int enable) {
  if (int rc = check_solver(s)) return rc;
  s->symmetric = enable != 0;
  return NS_OK;
}

int ns_timing_enable(ns_solver* s, int enable) {
  if (int rc = check_solver(s)) return rc;
  s->timing = enable != 0;
  return NS_OK;
}

int ns_timing_reset(ns_solver* s) {
  if (int rc = check_solver(s)) return rc;
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->timed.clear();
  s->pool_used = 0;
  return NS_OK;
}

int ns_timing_read(ns_solver* s, int kind, int64_t* launches, double* total_ms, double* flop) {
  if (int rc = check_solver(s)) return rc;
  HIP_TRY(hipStreamSynchronize(s->stream));
  int64_t cnt = 0;
  double ms = 0.0, fl = 0.0;
  for (const TimedLaunch& t : s->timed) {
    if (kind != 0 && t.kind != kind) continue;
    float e = 0.0f;
    HIP_TRY(hipEventElapsedTime(&e, t.beg, t.end));
    ++cnt;
    ms += e;
    fl += t.flop;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (flop) *flop = fl;
  return NS_OK;
}

int64_t ns_gemm_f64_partials(int64_t m, int64_t n, int flags) {
  if (m <= 0 || n <= 0) return 0;
  return gemm_f64_partials(m, n, (flags & NS_GEMM_SYMMETRIC) != 0);
}

size_t ns_gemm_f64_scratch_bytes(int64_t m, int64_t n, int64_t k, int flags) {
  return gemm_f64_split_bytes(m, n, k, (flags & NS_GEMM_SYMMETRIC) != 0);
}

int ns_gemm_f64(void* hip_stream, int64_t m, int64_t n, int64_t k, const double* X, int64_t ldx,
                const double* Y, int64_t ldy, double* D, int64_t ldd, const double* E1,
                int64_t lde1, const double* E2, int64_t lde2, double diag, double scale,
                int flags, double* sumsq_out) {
  return ns_gemm_f64_ws(hip_stream, m, n, k, X, ldx, Y, ldy, D, ldd, E1, lde1, E2, lde2, diag,
                        scale, flags, nullptr, 0, sumsq_out);
}

int ns_gemm_f64_ws(void* hip_stream, int64_t m, int64_t n, int64_t k, const double* X,
                   int64_t ldx, const double* Y, int64_t ldy, double* D, int64_t ldd,
                   const double* E1, int64_t lde1, const double* E2, int64_t lde2, double diag,
                   double scale, int flags, void* scratch, size_t scratch_bytes,
                   double* sumsq_out) {
  if (m < 0 || n < 0 || k < 0) return fail(NS_EINVAL, "negative size");
  if (flags & ~NS_GEMM_SYMMETRIC) return fail(NS_EINVAL, "unknown flags");
  if ((flags & NS_GEMM_SYMMETRIC) && m != n) return fail(NS_EINVAL, "symmetric output needs m == n");
  if (m == 0 || n == 0) return NS_OK;
  if (!D || (k > 0 && (!X || !Y))) return fail(NS_EINVAL, "null operand");
  if ((k > 0 && (ldx < k || ldy < n)) || ldd < n) return fail(NS_EINVAL, "leading dimension too small");
  if ((E1 && lde1 < n) || (E2 && lde2 < n)) return fail(NS_EINVAL, "addend leading dimension too small");
  if (D == X || D == Y) return fail(NS_EINVAL, "D must not alias X or Y");
  if (scratch && (reinterpret_cast<uintptr_t>(scratch) & 7))
    return fail(NS_EINVAL, "scratch must be 8-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  GemmF64Args a{};
  a.sk = scratch ? reinterpret_cast<double*>(scratch) : nullptr;
  a.sk_cap = scratch ? (int64_t)(scratch_bytes / sizeof(double)) : 0;
  a.X = X;
  a.Y = Y;
  a.D = D;
  a.E1 = E1;
  a.E2 = E2;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ldd = ldd;
  a.lde1 = lde1;
  a.lde2 = lde2;
  a.M = m;
  a.N = n;
  a.K = k;
  a.diag = diag;
  a.scale = scale;
  a.sym = (flags & NS_GEMM_SYMMETRIC) ? 1 : 0;
  // Per-tile partials live after the first element of sumsq_out.
  double* part = sumsq_out ? sumsq_out + 1 : nullptr;
  a.partial = part;
  const int64_t np = launch_gemm_f64(a, st);
  if (np < 0) return fail(NS_EHIP, "GEMM launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (sumsq_out) launch_reduce(part, np, sumsq_out, 0, 0.0, st);
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  return NS_OK;
}

int64_t ns_gemm_lp_partials(int64_t m, int64_t n) {
  if (m <= 0 || n <= 0) return 0;
  return gemm_lp_partials(m, n);
}

static int gemm_lp_entry(bool bf16, void* hip_stream, int64_t m, int64_t n, int64_t k,
                         const void* X, int64_t ldx, const void* Y, int64_t ldy, float* D,
                         int64_t ldd, uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1,
                         const float* E2, int64_t lde2, float diag, float scale,
                         double* sumsq_out) {
  if (m < 0 || n < 0 || k < 0) return fail(NS_EINVAL, "negative size");
  if (m == 0 || n == 0) return NS_OK;
  if ((!D && !Db) || (k > 0 && (!X || !Y))) return fail(NS_EINVAL, "null operand");
  const int64_t ycols = bf16 ? k : n;  // NT: Y is n x k
  if (k > 0 && (ldx < k || ldy < ycols)) return fail(NS_EINVAL, "leading dimension too small");
  if ((D && ldd < n) || (Db && lddb < n)) return fail(NS_EINVAL, "output leading dimension too small");
  if ((E1 && lde1 < n) || (E2 && lde2 < n)) return fail(NS_EINVAL, "addend leading dimension too small");
  if ((D && ((const void*)D == X || (const void*)D == Y)) ||
      (Db && ((const void*)Db == X || (const void*)Db == Y)))
    return fail(NS_EINVAL, "outputs must not alias X or Y");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  GemmLpArgs a{};
  a.X = X;
  a.Y = Y;
  a.D = D;
  a.Db = Db;
  a.E1 = E1;
  a.E2 = E2;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ldd = ldd;
  a.lddb = lddb;
  a.lde1 = lde1;
  a.lde2 = lde2;
  a.M = m;
  a.N = n;
  a.K = k;
  a.diag = diag;
  a.scale = scale;
  double* part = sumsq_out ? sumsq_out + 1 : nullptr;
  a.partial = part;
  const int64_t np = bf16 ? launch_gemm_bf16_nt(a, st) : launch_gemm_f32_nn(a, st);
  if (np < 0) return fail(NS_EHIP, "GEMM launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (sumsq_out) launch_reduce(part, np, sumsq_out, 0, 0.0, st);
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  return NS_OK;
}

int ns_gemm_f32(void* hip_stream, int64_t m, int64_t n, int64_t k, const float* X, int64_t ldx,
                const float* Y, int64_t ldy, float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                const float* E1, int64_t lde1, const float* E2, int64_t lde2, float diag,
                float scale, double* sumsq_out) {
  return gemm_lp_entry(false, hip_stream, m, n, k, X, ldx, Y, ldy, D, ldd, Db, lddb, E1, lde1, E2,
                       lde2, diag, scale, sumsq_out);
}

size_t ns_gemm_f32_split_scratch_bytes(int64_t m, int64_t n, int64_t k) {
  if (m < 0 || n < 0 || k < 0) return 0;
  return split_scratch_bytes(m, n, k);
}

// Argument checks shared by the split product's entry points.
static int split_args_ok(int64_t m, int64_t n, int64_t k, const float* X, int64_t ldx,
                         const float* Y, int64_t ldy, const float* D, int64_t ldd,
                         const uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1,
                         const float* E2, int64_t lde2) {
  if (m < 0 || n < 0 || k < 0) return fail(NS_EINVAL, "negative size");
  if (m == 0 || n == 0) return NS_OK;
  if ((!D && !Db) || (k > 0 && (!X || !Y))) return fail(NS_EINVAL, "null operand");
  if (k > 0 && (ldx < k || ldy < n)) return fail(NS_EINVAL, "leading dimension too small");
  if ((D && ldd < n) || (Db && lddb < n)) return fail(NS_EINVAL, "output leading dimension too small");
  if ((E1 && lde1 < n) || (E2 && lde2 < n)) return fail(NS_EINVAL, "addend leading dimension too small");
  if ((D && ((const void*)D == X || (const void*)D == Y)) ||
      (Db && ((const void*)Db == X || (const void*)Db == Y)))
    return fail(NS_EINVAL, "outputs must not alias X or Y");
  return NS_OK;
}

// The split product itself: operand splits into the planes of `sp`, the
// GEMM, and (sumsq_out non-NULL) the fixed-order reduction of the per-tile
// partial sums held at `part`.
static int split_gemm_run(hipStream_t st, int64_t m, int64_t n, int64_t k, const float* X,
                          int64_t ldx, const float* Y, int64_t ldy, float* D, int64_t ldd,
                          uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1,
                          const float* E2, int64_t lde2, float diag, float scale,
                          const SplitPlanes& sp, double* part, double* sumsq_out) {
  GemmLpArgs a{};
  if (k > 0) {
    split_operand(X, ldx, m, k, false, sp.xh, sp.xl, sp.ldk, sp.part, sp.exps, st);
    split_operand(Y, ldy, k, n, true, sp.yh, sp.yl, sp.ldk, sp.part + kSplitMaxParts,
                  sp.exps + 1, st);
    a.xexp = sp.exps;
    a.yexp = sp.exps + 1;
  }
  a.X = sp.xh;
  a.Xl = sp.xl;
  a.Y = sp.yh;
  a.Yl = sp.yl;
  a.ldx = a.ldy = sp.ldk;
  a.D = D;
  a.Db = Db;
  a.E1 = E1;
  a.E2 = E2;
  a.ldd = ldd;
  a.lddb = lddb;
  a.lde1 = lde1;
  a.lde2 = lde2;
  a.M = m;
  a.N = n;
  a.K = k;
  a.diag = diag;
  a.scale = scale;
  a.partial = sumsq_out ? part : nullptr;
  const int64_t np = launch_gemm_f16s_nt(a, st);
  if (np < 0) return fail(NS_EHIP, "GEMM launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (sumsq_out) launch_reduce(part, np, sumsq_out, 0, 0.0, st);
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  return NS_OK;
}

int ns_gemm_f32_split(void* hip_stream, int64_t m, int64_t n, int64_t k, const float* X,
                      int64_t ldx, const float* Y, int64_t ldy, float* D, int64_t ldd,
                      uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1, const float* E2,
                      int64_t lde2, float diag, float scale, double* sumsq_out, void* scratch,
                      size_t scratch_bytes) {
  const int rc = split_args_ok(m, n, k, X, ldx, Y, ldy, D, ldd, Db, lddb, E1, lde1, E2, lde2);
  if (rc != NS_OK || m == 0 || n == 0) return rc;
  if (!scratch || scratch_bytes < split_scratch_bytes(m, n, k))
    return fail(NS_ENOMEM, "scratch too small: %zu bytes needed", split_scratch_bytes(m, n, k));
  if ((reinterpret_cast<uintptr_t>(scratch) & (kAlign - 1)) != 0)
    return fail(NS_EINVAL, "scratch must be %zu-byte aligned", (size_t)kAlign);
  const SplitPlanes sp = carve_split(static_cast<char*>(scratch), m, n, k);
  return split_gemm_run(reinterpret_cast<hipStream_t>(hip_stream), m, n, k, X, ldx, Y, ldy, D,
                        ldd, Db, lddb, E1, lde1, E2, lde2, diag, scale, sp,
                        sumsq_out ? sumsq_out + 1 : nullptr, sumsq_out);
}

// ---- The split product without any allocation ----------------------------
// Scratch of ns_gemm_f32_split_noalloc: the split planes, block maxima and
// scale exponents, then the per-tile partial sums.  One copy per GPU, held by
// the loaded code object until the process ends.  In host code this name is
// not a device address; the address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char split_noalloc_scratch[NS_SPLIT_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// Device address of split_noalloc_scratch on the current device, looked up
// once per device (with that device current) and kept.
int noalloc_scratch(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(NS_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(split_noalloc_scratch)));
    if (!p) return fail(NS_EHIP, "hipGetSymbolAddress returned NULL");
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return NS_OK;
}

size_t noalloc_need(int64_t m, int64_t n, int64_t k, bool sumsq) {
  return split_scratch_bytes(m, n, k) +
         (sumsq ? align_up((size_t)gemm_lp_partials(m, n) * sizeof(double), kAlign) : 0);
}
}  // namespace

int ns_gemm_f32_split_noalloc(void* hip_stream, int64_t m, int64_t n, int64_t k,
                              const float* X, int64_t ldx, const float* Y, int64_t ldy,
                              float* D, int64_t ldd, uint16_t* Db, int64_t lddb,
                              const float* E1, int64_t lde1, const float* E2, int64_t lde2,
                              float diag, float scale, double* sumsq_out) {
  const int rc = split_args_ok(m, n, k, X, ldx, Y, ldy, D, ldd, Db, lddb, E1, lde1, E2, lde2);
  if (rc != NS_OK || m == 0 || n == 0) return rc;
  const size_t need = noalloc_need(m, n, k, sumsq_out != nullptr);
  if (need > (size_t)NS_SPLIT_NOALLOC_MAX_BYTES)
    return fail(NS_ENOMEM,
                "shape %lld x %lld x %lld needs %zu bytes of scratch; the built-in "
                "scratch holds %zu (use ns_gemm_f32_split with a workspace)",
                (long long)m, (long long)n, (long long)k, need,
                (size_t)NS_SPLIT_NOALLOC_MAX_BYTES);
  void* base = nullptr;
  const int rs = noalloc_scratch(&base);
  if (rs != NS_OK) return rs;
  char* p = static_cast<char*>(base);
  const SplitPlanes sp = carve_split(p, m, n, k);
  double* part = reinterpret_cast<double*>(p + split_scratch_bytes(m, n, k));
  return split_gemm_run(reinterpret_cast<hipStream_t>(hip_stream), m, n, k, X, ldx, Y, ldy, D,
                        ldd, Db, lddb, E1, lde1, E2, lde2, diag, scale, sp, part, sumsq_out);
}

// The symmetric-output bf16 kernel faulted the GPU on its first test and the
// fault's cause has not been found, so the path is switched off: the flag is
// rejected and the solver runs every bf16 product in full.
constexpr bool kBf16SymEnabled = false;

size_t ns_gemm_bf16_scratch_bytes(int64_t m, int64_t n, int64_t k, int flags) {
  if (!kBf16SymEnabled) return 0;
  if (m <= 0 || n <= 0 || k < 0 || m != n || !(flags & NS_GEMM_SYMMETRIC)) return 0;
  return (size_t)gemm_bf16_sym_scratch_floats(n, k) * sizeof(float);
}

int ns_gemm_bf16_nt_ws(void* hip_stream, int64_t m, int64_t n, int64_t k, const uint16_t* X,
                       int64_t ldx, const uint16_t* Y, int64_t ldy, float* D, int64_t ldd,
                       uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1, const float* E2,
                       int64_t lde2, float diag, float scale, int flags, double* sumsq_out,
                       void* scratch, size_t scratch_bytes) {
  if (!(flags & NS_GEMM_SYMMETRIC))
    return gemm_lp_entry(true, hip_stream, m, n, k, X, ldx, Y, ldy, D, ldd, Db, lddb, E1, lde1,
                         E2, lde2, diag, scale, sumsq_out);
  if (flags & ~NS_GEMM_SYMMETRIC) return fail(NS_EINVAL, "unknown flags %d", flags);
  if (!kBf16SymEnabled)
    return fail(NS_EINVAL, "the symmetric-output bf16 kernel is disabled");
  if (m != n) return fail(NS_EINVAL, "a symmetric output needs m == n");
  if (m < 0 || k < 0) return fail(NS_EINVAL, "negative size");
  if (m == 0) return NS_OK;
  if ((!D && !Db) || (k > 0 && (!X || !Y))) return fail(NS_EINVAL, "null operand");
  if (k > 0 && (ldx < k || ldy < k)) return fail(NS_EINVAL, "leading dimension too small");
  if ((D && ldd < n) || (Db && lddb < n)) return fail(NS_EINVAL, "output leading dimension too small");
  if ((E1 && lde1 < n) || (E2 && lde2 < n)) return fail(NS_EINVAL, "addend leading dimension too small");
  if ((D && ((const void*)D == X || (const void*)D == Y)) ||
      (Db && ((const void*)Db == X || (const void*)Db == Y)))
    return fail(NS_EINVAL, "outputs must not alias X or Y");
  const size_t need = ns_gemm_bf16_scratch_bytes(m, n, k, flags);
  if (need > 0 && (!scratch || scratch_bytes < need))
    return fail(NS_ENOMEM, "scratch too small: %zu bytes needed", need);
  if (scratch && (reinterpret_cast<uintptr_t>(scratch) & 15) != 0)
    return fail(NS_EINVAL, "scratch must be 16-byte aligned");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  GemmLpArgs a{};
  a.X = X;
  a.Y = Y;
  a.D = D;
  a.Db = Db;
  a.E1 = E1;
  a.E2 = E2;
  a.ldx = ldx;
  a.ldy = ldy;
  a.ldd = ldd;
  a.lddb = lddb;
  a.lde1 = lde1;
  a.lde2 = lde2;
  a.M = m;
  a.N = n;
  a.K = k;
  a.diag = diag;
  a.scale = scale;
  double* part = sumsq_out ? sumsq_out + 1 : nullptr;
  a.partial = part;
  int64_t np = launch_gemm_bf16_sym(a, static_cast<float*>(scratch),
                                    (int64_t)(scratch_bytes / sizeof(float)), st);
  if (np == -2) np = launch_gemm_bf16_nt(a, st);   // shape served by the full-output kernel
  if (np < 0) return fail(NS_EHIP, "GEMM launch failed: %s", hipGetErrorString(hipGetLastError()));
  if (sumsq_out) launch_reduce(part, np, sumsq_out, 0, 0.0, st);
  if (hipGetLastError() != hipSuccess) return fail(NS_EHIP, "kernel launch failed");
  return NS_OK;
}

int ns_gemm_bf16_nt(void* hip_stream, int64_t m, int64_t n, int64_t k, const uint16_t* X,
                    int64_t ldx, const uint16_t* Y, int64_t ldy, float* D, int64_t ldd,
                    uint16_t* Db, int64_t lddb, const float* E1, int64_t lde1, const float* E2,
                    int64_t lde2, float diag, float scale, double* sumsq_out) {
  return gemm_lp_entry(true, hip_stream, m, n, k, X, ldx, Y, ldy, D, ldd, Db, lddb, E1, lde1, E2,
                       lde2, diag, scale, sumsq_out);
}

}  // extern "C"
