// Leading spectrum of the transfer matrix of a CTMRG environment.
#pragma once
#include "engine.hpp"

namespace ctm {

class Transfer {
 public:
  // direction 0: one column (T1, a, T3); 1: one row (T2, a rotated, T4);
  // site = false leaves the site tensor out.
  Transfer(Env& env, int direction, bool site);
  // Ritz values of `krylov` Arnoldi steps (at most 64 and the dimension)
  // from a seeded random start, unsorted; returns their number.
  int spectrum(int krylov, unsigned long long seed, double* wr, double* wi);
  size_t dim = 0;

 private:
  void apply(const double* v, double* out);
  Env& e;
  Context& ctx;
  int direction;
  bool site;
  int chi, d;
  DevBuf w1, w2, aT;
  SliceCache aslices;  // BF16 slices of aT (reduced-precision modes)
};

}  // namespace ctm
