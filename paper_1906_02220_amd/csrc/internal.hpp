// Internal declarations of the CTMRG library: error handling, the context,
// and the launchers of the hand-written gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>
#include <functional>
#include <map>
#include <tuple>

namespace ctm {

// Error carrying one of the CTM_* status codes; converted at the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define CTM_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      throw ::ctm::Error(-3, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

#define CTM_REQUIRE(cond, msg)                                                     \
  do {                                                                             \
    if (!(cond)) throw ::ctm::Error(-1, msg);                                      \
  } while (0)

// Debugging aid: while set, every device buffer the library allocates is
// filled with all-ones bytes (a NaN as a double, -1 as an int) before use, so
// that a kernel reading memory the library never wrote gives NaN or garbage
// instead of whatever the allocator handed back (often zeros in a fresh
// process, earlier results in a long-running one), and sits between two
// guard bands of kGuardBytes with a fixed byte pattern that release() checks,
// so that a kernel writing past either end of a buffer is reported.  Starts
// from the environment variable CTM_POISON_ALLOC (set and not "0": on).
std::atomic<int>& poison_allocations();
constexpr size_t kGuardBytes = 64 * 1024;
// hipMalloc of nbytes between guard bands (poisoned) or plain; returns the
// user pointer, or nullptr on failure
void* debug_malloc(size_t nbytes, bool guarded);
// frees a debug_malloc pointer; a guarded one has its bands checked first
// (waiting for the device) and a damaged band counted and reported on stderr
void debug_free(void* p, size_t nbytes, bool guarded);
// damaged guard bands found so far
long long guard_violations();

// Device buffer of doubles (or raw bytes) owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool guarded = false;  // allocated between guard bands (poisoning on)
  DevBuf() = default;
  explicit DevBuf(size_t nbytes) { alloc(nbytes); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), guarded(o.guarded) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      guarded = o.guarded;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t nbytes) {
    release();
    if (nbytes == 0) return;
    const bool g = poison_allocations().load(std::memory_order_relaxed) != 0;
    p = debug_malloc(nbytes, g);
    if (!p) {
      (void)hipGetLastError();
      throw Error(-2, "hipMalloc of " + std::to_string(nbytes) + " bytes failed");
    }
    bytes = nbytes;
    guarded = g;
  }
  void release() {
    if (p) debug_free(p, bytes, guarded);
    p = nullptr;
    bytes = 0;
    guarded = false;
  }
  double* d() const { return static_cast<double*>(p); }
  float* f() const { return static_cast<float*>(p); }
};

// Accumulated event timing per kernel class.
struct TimingClass {
  long long count = 0;
  double ms = 0.0;
  double flops = 0.0;
};

struct Context {
  int device = 0;
  int num_cus = 256;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  std::string last_error;
  bool timing = false;
  bool use_graphs = false;  // replay warm sweeps from captured HIP graphs
  bool autotune = false;    // time the kernel variants of each product shape once
  // fastest variant per (kind, M, N, K, timing class)
  std::map<std::tuple<int, int, int, int, int>, int> tuned;
  TimingClass tcls[3];
  // events pending resolution: (class, start, stop, flops)
  struct Pending { int cls; hipEvent_t a, b; double flops; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  DevBuf splitk_ws;     // split-K partial products
  DevBuf mixed_ws;      // operand slices and scales of the reduced-precision GEMMs
  DevBuf scratch_small; // reductions and flags
  DevBuf jacobi_ws;     // rotation log, ranks and sweep count of the Jacobi SVD
  // When set, the split-K partials of gemm_f64 and the reduction partials go
  // to this caller-provided device memory instead of the workspaces above,
  // and a product whose partials do not fit is refused: nothing is allocated.
  double* fixed_splitk = nullptr;
  size_t fixed_splitk_bytes = 0;
  double* fixed_red = nullptr;  // at least kRedScratchDoubles
  Context() = default;
  Context(const Context&) = delete;
  Context& operator=(const Context&) = delete;
  ~Context();
  hipEvent_t get_event();
  void resolve_timing();
};

// Scoped timer: records an event pair around a region when timing is on.
struct ScopedTimer {
  Context& c;
  int cls;
  double flops;
  hipEvent_t a = nullptr, b = nullptr;
  ScopedTimer(Context& ctx, int cls_, double fl) : c(ctx), cls(cls_), flops(fl) {
    if (c.timing && cls >= 0) { a = c.get_event(); CTM_HIP(hipEventRecord(a, c.stream)); }
  }
  ~ScopedTimer() {
    if (c.timing && a) {
      b = c.get_event();
      if (hipEventRecord(b, c.stream) == hipSuccess) c.pending.push_back({cls, a, b, flops});
    }
  }
};

// Tile of a workgroup, XCD-aware.  Workgroups are dispatched round-robin
// over the 8 XCDs (workgroup w runs on XCD w % 8), and each XCD has its own
// L2.  Tile t = (w % 8) * (T / 8) + ... gives every XCD a contiguous range of
// the tile order, and that order walks G tile rows at a time, so one XCD
// touches about G row panels of A and range / G column panels of B instead
// of all of them.
template <int G>
__device__ inline void xcd_tile(int w, int ntm, int ntn, int& tm, int& tn) {
  const int T = ntm * ntn;
  const int x = w & 7, loc = w >> 3;
  const int t = x * (T >> 3) + min(x, T & 7) + loc;
  const int grp = t / (G * ntn);
  const int first = grp * G;
  const int gs = min(ntm - first, G);
  const int r = t - grp * G * ntn;
  tm = first + r % gs;
  tn = r / gs;
}

// ---------------------------------------------------------------- matrices

// A strided matrix view: element (i, j) of batch z is at
// ptr[z * bs + i * rs + j * cs].
struct View {
  const double* p;
  long long rs, cs, bs;
};
struct ViewOut {
  double* p;
  long long rs, cs, bs;
};

inline View rowmajor(const double* p, long long ld, long long bs = 0) { return {p, ld, 1, bs}; }
inline View colmajor(const double* p, long long ld, long long bs = 0) { return {p, 1, ld, bs}; }
inline ViewOut out_rowmajor(double* p, long long ld, long long bs = 0) { return {p, ld, 1, bs}; }

// Variant of a product shape to launch: 0 unless the context autotunes; then
// the first call of each (kind, M, N, K, cls) runs every variant once to warm
// up and twice more between events, keeps the fastest, and later calls reuse
// it.  run(v) launches variant v on ctx.stream; all variants of a kind must
// compute the same result (the same K order per output element).
int pick_variant(Context& ctx, int kind, int M, int N, int K, int cls, int nvariants,
                 const std::function<void(int)>& run);

// C = alpha * A(MxK) * B(KxN) + beta * C, FP64 MFMA, for `batch` matrices.
// `cls` selects the timing class (-1: time only under class 1).
void gemm_f64(Context& ctx, int M, int N, int K, double alpha, View A, View B, double beta,
              ViewOut C, int batch = 1, int cls = -1);

// Contraction in the precision mode of ctm.h (CTM_PREC_*) with FP64 inputs
// and outputs: FP32 MFMA for CTM_PREC_F32, BF16 slices for CTM_PREC_BF16X*.
// Products the reduced-precision kernels do not cover (alpha != 1, beta != 0,
// batched or transposed operands) and CTM_PREC_F64 run as gemm_f64.
// Grouped products C = A B: independent problems run in one persistent
// launch whose workgroups claim tiles from a device counter (see
// dgemm_rr_grouped).  A problem is grouped only where the plain call would
// run the same tile kernel without split-K, so that grouping never changes
// a result.
struct GroupProblem {
  const double* A;
  const double* B;
  double* C;
  int M, N, K, lda, ldb, ldc;
};
constexpr int kGroupMax = 32;
struct GroupTable {
  int count, total;
  int tile_start[kGroupMax + 1];
  GroupProblem p[kGroupMax];
};
// dgemm_rr without split-K would take this product
bool rr_grouped_ok(const Context& ctx, int M, int N, int K, View A, View B, ViewOut C);
void gemm_grouped_f64(Context& ctx, const GroupTable& tab, int* counter);
// 1: the product of `mode` runs on the FP64 96 x 96 kernel, 2: on the FP32
// 96 x 96 kernel (both without split-K), 0: on neither (it is not grouped)
int grouped_kind(const Context& ctx, int mode, int M, int N, int K, View A, View B, ViewOut C);
// all problems of one kind, in launches of at most kGroupMax problems on
// ctx.stream; counter: one int of device memory
void gemm_grouped(Context& ctx, int kind, const GroupProblem* probs, int count, int* counter);

void gemm_mixed(Context& ctx, int mode, int M, int N, int K, double alpha, View A, View B,
                double beta, ViewOut C, int batch = 1, int cls = -1);
// Modes gemm_mixed implements.
bool mixed_mode_supported(int mode);

// Where a product writes element (i, j): C[(i / r2) sr1 + (i % r2) sr2 +
// (j / c2) sc1 + j % c2], i.e. rows and columns each split into two indices,
// so that a permutation that keeps the last column index innermost can be
// written by the product itself.  plain(M, N, ldc) is the row-major layout.
struct OutMap {
  int r2;
  long long sr1, sr2;
  int c2;
  long long sc1;
  static OutMap plain(int M, int N, long long ldc) { return OutMap{M, 0, ldc, N, 0}; }
  __host__ __device__ long long at(int i, int j) const {
    return (long long)(i / r2) * sr1 + (long long)(i % r2) * sr2 + (long long)(j / c2) * sc1 + j % c2;
  }
};
// The slices and column maxima of a B operand that stays constant over many
// products (the rotated site tensor): filled by the first product that uses
// it, reused while `valid` (the owner clears it when B changes).
struct SliceCache {
  DevBuf q, mx;
  int S = 0, N = 0, K = 0;
  const void* src = nullptr;
  bool valid = false;
};
// C = A B through `om` when `mode` is a BF16 slice mode and the slice kernel
// covers the product (returns true); otherwise nothing runs and it returns
// false, and the caller takes the plain path.  With bc, B's slices come from
// (or go to) that cache.
bool gemm_slices_split_out(Context& ctx, int mode, int M, int N, int K, View A, View B, double* C,
                           const OutMap& om, int cls = -1, SliceCache* bc = nullptr);

// out = permutation of `in` (row-major dims[0..rank-1]); out axis a is in
// axis perm[a].  rank <= 8.
void permute(Context& ctx, const double* in, double* out, int rank, const long long* dims,
             const int* perm);

// ---------------------------------------------------------------- small kernels

// Doubles of reduction scratch the two-stage reductions use.
constexpr size_t kRedScratchDoubles = 512 + 64;

void fill_zero(Context& ctx, double* p, size_t n);
void fill_zero_int(Context& ctx, int* p, size_t n);
// Lets `fn` launch with `bytes` of dynamic LDS (above the 64 KB default, up
// to the 160 KB of a gfx950 CU); a no-op after the first call per size.
void allow_lds(const void* fn, size_t bytes);
void copy_dev(Context& ctx, double* dst, const double* src, size_t n);
// dst[i * ldd + j] = src[i * lds + j] for i < rows, j < cols (row-major blocks).
void copy_block(Context& ctx, double* dst, long long ldd, const double* src, long long lds,
                int rows, int cols);
// p /= max|p|; *log_slot += log(max|p|); *flag = 1 if p is not finite or all zero.
// If inv_keep is not null, *inv_keep receives the factor 1/max|p| applied.
void normalise_maxabs(Context& ctx, double* p, size_t n, double* log_slot, int* flag,
                      double* inv_keep = nullptr);
// *result = sum x[i] * y[i] (fixed-order two-stage reduction, deterministic)
void dot(Context& ctx, const double* x, const double* y, size_t n, double* result);
// Fill count doubles with standard normal numbers from the counter-based
// generator (SplitMix64 mixing of seed and element counter, Box-Muller).
void fill_normal(Context& ctx, double* Z, size_t count, unsigned long long seed,
                 unsigned long long counter);
// From the b x b Gram matrix G = Z^T Z of an n x b block Z (b <= 128):
// W = D^-1 R^-1 with D = sqrt(diag G) and R^T R = D^-1 G D^-1 (upper R), so
// that Z W has orthonormal columns.  A column whose Schur-complement pivot
// falls below dep_tol is dependent: it takes no part in the elimination and
// dep[j] = 1 (its column of Z W must be replaced).  *err = 1 on non-finite G.
// With first_order (for the second pass of a CholeskyQR): when
// max |G - I| <= kNearIdentityTol, W = (3 I - G) / 2 instead (Z W is then
// orthonormal to O(|G - I|^2)) and no column is dependent; the kernel decides
// on the device and skips the factorisation.
constexpr double kNearIdentityTol = 1e-10;
void chol_inverse(Context& ctx, const double* G, int b, double dep_tol, double* W, int* dep,
                  int* err, bool first_order = false);
// Replace the columns j with dep[j] != 0 of an n x b row-major Q by standard
// normal numbers from the counter-based generator, starting at the counter
// *counter_in (device memory); *counter_out (another device slot) receives
// the counter advanced by n * b.  Keeping the counter on the device makes a
// replayed graph draw the same numbers as the eager run it was captured from.
void refill_columns(Context& ctx, double* Q, int ldq, int n, int b, const int* dep,
                    unsigned long long seed, const unsigned long long* counter_in,
                    unsigned long long* counter_out);
// One-sided Jacobi SVD of a b x b row-major matrix B = X diag(s) Y^T (b <= 128),
// singular values sorted descending.  X and Y (b x b row-major) may be null
// when only the values are wanted; vectors are computed for one matrix per
// call (batch = 1), values for batch matrices at stride bstride.  With
// trans the rotations act on the columns of B^T (faster for a graded upper
// triangular B).  With zr > 0, pairs with a column of norm at most
// zr ||B||_F (zero to working precision for zr ~ b eps) do not keep the
// sweeps going; with zp > 0, neither do pairs whose two columns are both at
// most zp ||B||_F (B known to a relative accuracy zp).  *err = 1 if the
// sweeps did not converge or produced non-finite values.
void jacobi_svd(Context& ctx, const double* B, int b, double* X, double* s, double* Y, int* err,
                int batch = 1, long long bstride = 0, long long sstride = 0, bool trans = false,
                double zr = 0.0, double zp = 0.0);
// Maximum b supported by jacobi_svd with vectors / values only.
int jacobi_max_b(bool vectors);
// out[i] = ||Y[:, i] - s[i] V[:, i]||_2 for i < kk (Y, V: n rows, leading
// dimension ld, row-major), then out[kk] = s[0].
void column_residuals(Context& ctx, const double* Y, const double* V, const double* s, int n,
                      int ld, int kk, double* out);
// w[j] = 1/sqrt(s[j]) if j < kk and s[j] > eps * s[0] > 0, else 0; j < chi.
void inv_sqrt_cut(Context& ctx, const double* s, int kk, int chi, double eps, double* w);
// Z[i][j] *= w[j] for an n x c block of a row-major matrix with leading dim ldz.
void scale_cols(Context& ctx, double* Z, int n, int c, int ldz, const double* w);
// Flip the signs of column j of X and Y (n rows, b columns) so that the entry
// of largest magnitude of X[:, j] is positive (ties: lowest row).
void fix_signs(Context& ctx, double* X, int ldx, double* Y, int ldy, int n, int b);
// For 4 spectra s (4 x chi, each descending): s_hat = s / ||s||_2 per corner;
// *delta = max_c ||s_hat_c - old_c||_2; old <- s_hat.
void spectra_delta(Context& ctx, const double* s, double* old, int chi, double* delta);

}  // namespace ctm
