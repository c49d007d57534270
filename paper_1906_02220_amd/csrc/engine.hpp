// CTMRG engine: environment state and the orchestration of the absorption
// moves, sweeps and observables on one GPU.
#pragma once
#include "internal.hpp"

namespace ctm {

struct EnvOptions {
  int precision = 0;
  double eps_cut = 1e-12;
  int svd_block = 0;
  int svd_iters = 0;
  int svd_iters_cold = 0;
  int svd_oversample = 0;
  // > 0: after the Rayleigh-Ritz step, iterate again (from its vectors) until
  // the largest residual ||Mt^T u_i - s_i v_i|| / s_1 of the kept triplets is
  // at most svd_tol; <= 0: the fixed iteration counts only
  double svd_tol = 0.0;
  int move_order[4] = {0, 2, 1, 3};  // directions of a sweep: left, right, up, down
  unsigned long long seed = 0x5eedULL;
  std::vector<double> boundary;  // empty: default
};

class Grad;
class Transfer;

// Per-move record of the forward pass kept for the adjoint: the environment
// before the move, the kept singular triplets of the cut matrix and the
// normalisation factors of the three renormalised tensors.
struct TapeLayout {
  size_t c, t, ua, va, s, w, inv, total;
  TapeLayout(int chi, int d) {
    const size_t n = (size_t)chi * d;
    c = 0;
    t = c + 4ull * chi * chi;
    ua = t + 4ull * chi * d * chi;
    va = ua + n * chi;
    s = va + n * chi;
    w = s + chi;
    inv = w + chi;
    total = inv + 4;
  }
};

class Env {
  friend class Grad;
  friend class Transfer;

 public:
  Env(Context& ctx, int d, int chi, const EnvOptions& opt);
  ~Env();
  Env(const Env&) = delete;
  Env& operator=(const Env&) = delete;
  // classical / user site tensor (device pointer, d^4)
  void set_site_tensor_dev(const double* a_dev);
  // purification pair (device pointers [2][2][x][y][z])
  void build_purification_dev(const double* A, const double* B, int D, int D_gamma, int gamma);
  void init_boundary();

  void move(int k);              // left move in the frame rotated k times
  // The three parts of move(k), for batches run in lock-step: the tape record
  // and the enlarged corners; the two half-system products and the cut matrix
  // (a5); the projectors and the absorption (a6, a7).
  void move_front(int k);
  void move_products(int k);
  void move_back(int k);
  // The products of move_products(k) as grouped problems: U and Lt (independent)
  // in probs[0..1], then Mt = Lt U in probs[2].  Returns the kernel kind of
  // grouped_kind, or 0 if this environment has to run them itself.
  int cut_products(int k, GroupProblem* probs);
  // The rest of a sweep after its four moves: corner spectra and delta, then
  // the copies to pinned host memory that sweep_finish reads.  Drops a
  // captured sweep graph (the next graph-enabled sweep captures a new one).
  void sweep_tail_eager();
  int sweep(int max_sweeps, double tol, int* done, double* delta);
  // One sweep without waiting for it: the four moves and the corner-spectrum
  // delta (replayed from a captured HIP graph when the context allows graphs
  // and the previous sweep was a warm one), then asynchronous copies of the
  // delta and the error flags to pinned host memory.
  void sweep_enqueue();
  // After ctx.stream has drained: the delta of that sweep; throws on a
  // numerical failure the kernels flagged.
  double sweep_finish(const char* where);

  double kappa();
  void log_z(double* log_abs, double* sign);
  void bond_metric(double* host_out, size_t len);
  // Unnormalised ring E of a purification environment reordered to
  // [ket u,l,d,r][bra u,l,d,r] (D^4 x D^4), written to device memory.
  void ring_ket_bra_dev(double* out);
  const double* composite_dev() const { return Kc.d(); }  // 16 x D^4
  double expect_op(const double* op, int op_dim);
  // expect_op on the current ring with every device buffer taken from
  // `scratch` (scratch_doubles doubles of device memory): nothing is
  // allocated.  Refused when the ring is not current or D is too large.
  double expect_op_fixed(const double* op, int op_dim, double* scratch, size_t scratch_doubles);
  size_t expect_scratch_doubles() const;
  double expect_tensor(const double* a_imp_host);
  void corner_spectra(double* host_out, size_t len);
  void get(double* C, double* T, double* logs);
  void set(const double* C, const double* T, const double* logs);
  // max_i ||Mt^T u_i - s_i v_i|| / s_1 over the kept triplets of the last
  // move's truncated SVD (0 before the first move)
  double last_svd_residual();
  // truncated SVDs by subspace iteration so far and their iterations
  long long svd_calls = 0, svd_iterations = 0;

  Context& ctx;
  int d, chi, n;
  int D = 0;          // 0: not a purification environment
  int sweeps_done = 0;
  EnvOptions opt;
  int b = 0;          // subspace size of the projector SVD
  // When set, move() writes its TapeLayout record here (device memory).
  double* tape_slot = nullptr;

 private:
  void alloc();
  void sweep_body();
  bool graph_ready() const;
  void capture_graph();
  void drop_graph();
  void corner(int f);
  void svd_top(const double* Mt, int k);
  void subspace_iteration(const double* Mt);
  void rayleigh_ritz(const double* Mt);
  void final_iteration_ritz(const double* Mt);
  double svd_residual(const double* Mt);
  void orth(double* Z, double* Q, int passes);
  void ring();
  double expect_from_ring(const double* O, const double* I16, double* F, double* rhoT, double* dO,
                          double* dI);
  void reset_spectra();
  void check_flags(const char* where);
  const double* Cp(int i) const { return Call.d() + (size_t)(i & 3) * chi * chi; }
  double* Cw(int i) { return Call.d() + (size_t)(i & 3) * chi * chi; }
  const double* Tp(int i) const { return Tall.d() + (size_t)(i & 3) * chi * d * chi; }
  double* Tw(int i) { return Tall.d() + (size_t)(i & 3) * chi * d * chi; }

  DevBuf arot[4];
  SliceCache aslices[4];    // BF16 slices of arot[f], valid until the site tensor changes
  DevBuf Kc;                // composite 16 x D^4
  DevBuf Call, Tall;        // 4 chi^2, 4 chi^2 d
  DevBuf logs;              // 8 log scales
  DevBuf Qb[4], X1[4];
  bool qvalid[4] = {false, false, false, false};
  DevBuf U, Lt, Mt, t1, t2;
  DevBuf Om, Zb, Z0, Qz, Wv, G, Wm, Bsm, xs, ys, sv, UA, VA, winv, Pu, Pl, sm1, sm2, sm3;
  DevBuf warm[4];
  bool warm_ok[4] = {false, false, false, false};
  // Warm moves per direction since its last cold start, counted up to
  // kSettleWarmMoves.  With the automatic iteration count (svd_iters_auto)
  // the first kSettleWarmMoves warm moves of a direction run two subspace
  // iterations, later ones opt.svd_iters (one).
  static constexpr int kSettleWarmMoves = 8;
  int warm_moves[4] = {0, 0, 0, 0};
  bool svd_iters_auto = false;
  DevBuf spec_s, spec_old, scal;  // scal: delta and observables scalars
  DevBuf iflags;                  // [0] numeric, [1] svd, [8..] dependency flags
  DevBuf E, E8;
  DevBuf resid;                   // column residuals of the truncated SVD, then s_1
  double* hres = nullptr;         // pinned host copy of resid
  bool moved = false;             // a move has run: Mt, UA, VA, sv are its own
  bool e_valid = false;
  unsigned long long rng_ctr = 0;  // counter of the cold-start draws
  DevBuf rngc;                     // two device slots of the refill counter
  int rng_slot = 0;                // slot the next refill reads
  // graph of one warm sweep and the context workspaces it was captured with
  hipGraphExec_t gexec = nullptr;
  const void* g_splitk = nullptr;
  const void* g_mixed = nullptr;
  bool warm_eager_done = false;  // a warm sweep ran eagerly (workspaces sized)
  double* hbox = nullptr;        // pinned host memory: delta, then two int flags
};

}  // namespace ctm
