// Full-update truncation of a gated bond in the CTMRG environment.
#pragma once
#include "engine.hpp"

namespace ctm {

class FullUpdate {
 public:
  FullUpdate(Context& ctx, int D, int gamma);
  // A, B, A_out, B_out: host [2][2][D][D][D]; H host 4 x 4; errors host,
  // als_iters + 1 entries (may be null).
  void run(const double* A, const double* B, const double* H, double tau, int chi,
           const EnvOptions& opt, int sweeps, int als_iters, double* A_out, double* B_out,
           double* errors);

 private:
  void fused(const double* in, double* out, bool back);
  void composite(const double* Afused, const double* Bfused, double* K);
  double error(const double* Afused, const double* Bfused);
  void solve(int side);

  Context& ctx;
  int D, gamma;
  double normK = 1.0;
  DevBuf A0, B0, Ap, Bp, Acur, Bcur, Ag, Bg, Hd, Gd, gs, X, Y, sv;
  DevBuf E, Es, Kg, KE, KEt, dK, M, P, Nm, rhs, Kraw, scal, flag;
};

}  // namespace ctm
