// Reverse-mode derivative of the CTMRG environment: the gradient of
// L = w_k ln(kappa) + w_o <O> with respect to the site tensor, and through the
// double layer and the composite to the purification tensors A and B.
#pragma once
#include "engine.hpp"

namespace ctm {

struct GradStats {
  int moves = 0;
  int cg_iters_max = 0;
  long long cg_iters_total = 0;
  double ms_forward = 0.0, ms_recompute = 0.0, ms_backward = 0.0;
  double tape_bytes = 0.0, checkpoint_bytes = 0.0;
};

class Grad {
 public:
  // sweeps fixed sweeps from the environment's current state; the state is
  // checkpointed every ckpt_every sweeps (<= 0: one segment).
  Grad(Env& env, int sweeps, int ckpt_every);
  void forward();
  // Loss at the final state and the adjoint seeds.  For a purification
  // environment op (op_dim 4 or 16) defines <O>; otherwise a_imp (d^4 host
  // array) defines <O> = <E, a_imp> / <E, a>.  Either may be null if w_o = 0.
  double seed(double w_k, double w_o, const double* op, int op_dim, const double* a_imp,
              double* log_kappa, double* expect);
  void backward();
  // dL/da, a[u][l][d][r] (device, d^4), written on ctx.stream
  void grad_site(double* ga_dev);
  // dL/dA, dL/dB in the layout of the inputs (device arrays of 4 D^2 D_gamma
  // each, read and written on ctx.stream)
  void grad_purification(const double* A_dev, const double* B_dev, int D, int Dg, int gamma,
                         double* gA_dev, double* gB_dev);
  GradStats stats;

 private:
  struct Ckpt {
    DevBuf C, T, logs, warm, rng;
    bool warm_ok[4];
    int warm_moves[4];
    int rng_slot;
    unsigned long long rng_ctr;
  };
  void save(Ckpt& c);
  void restore(const Ckpt& c);
  void run_segment(int sg, bool record);
  void move_bwd(int k, const double* rec);
  void svd_bwd(const double* UA, const double* VA, const double* s, const double* w);
  int cg(const double* UA, const double* s);
  void site_total();

  Env& e;
  Context& ctx;
  int sweeps, every, nseg;
  int chi, d, n;
  TapeLayout tl;
  std::vector<Ckpt> ck;
  DevBuf tape;
  // adjoints
  DevBuf Cb, Tb, arb[4], abar, Kcb;
  // n^2 (or d^4) work; [Mt^T | Mt | Mt^T]; transposed rotated site tensors
  DevBuf Qbar, wA, wB, Mt3, arotT[4];
  // n x chi work, n x 2 chi factors of the half-system adjoints
  DevBuf PuU, PlU, Pub, Plb, UAw, VAw, UAb, VAb, x1e, G1T, G2, pb, sm1b, X1b;
  DevBuf LU, RU, LL, RL, Wf;
  // conjugate gradients: both systems stacked (n chi apart)
  DevBuf cgX, cgR, cgP, cgAP, cgXb, cgT;
  // chi x chi and smaller
  DevBuf ckb, cq3b, tq3b, sm2b, Gu, Gv, Zm, tmpA, tmpB, wbar, sbar;
  DevBuf rr, bn, best, stall, active, count;
  int* hcount = nullptr;  // pinned host copy of the active-column count
  bool site_done = false;
};

}  // namespace ctm
