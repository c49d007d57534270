// Index permutation of row-major FP64 tensors (rank <= 8).
//
// When the innermost axis stays innermost, every thread copies one element
// with both reads and writes contiguous along that axis.  Otherwise the
// kernel transposes tiles of the plane spanned by the input's innermost axis
// P (contiguous in the input) and the input axis Q that becomes innermost in
// the output (contiguous in the output) through LDS, so both the global
// reads and the global writes are coalesced; all remaining axes enumerate
// the tiles' batch.  A tile spans the whole plane when it is small (P up to
// 128, Q up to 64, at most kTileElems elements), so that planes such as the
// 72 x 36 one of an edge tensor's [chi, d, d, chi] -> [chi, chi, d, d]
// permutation move as one dense tile instead of six 32 x 32 tiles that are
// 42 % full.
#include "internal.hpp"

namespace ctm {

namespace {

struct PermDesc {
  int rank;                // number of axes after merging
  long long odim[8];       // output dims
  long long istr[8];       // input stride of output axis a
  long long ostr[8];       // output stride of output axis a
};

__global__ void permute_copy_kernel(const double* __restrict__ in, double* __restrict__ out,
                                    PermDesc pd, long long total) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    long long rem = idx, off = 0;
    for (int a = pd.rank - 1; a >= 0; --a) {
      const long long q = rem / pd.odim[a];
      off += (rem - q * pd.odim[a]) * pd.istr[a];
      rem = q;
    }
    out[idx] = in[off];
  }
}

// Tiled transpose.  Axis P: input innermost (input stride 1), output axis ap;
// axis Q: output innermost (output stride 1), input stride qs.  The other
// output axes (up to 6) index the batch.
struct TDesc {
  long long dimP, dimQ;
  long long qs_in;       // input stride of Q
  long long ps_out;      // output stride of P
  int nb;                // number of batch axes
  long long bdim[8], bin[8], bout[8];
  long long tilesP, tilesQ;
  int TP, TQ;            // tile extent along P and Q
};

constexpr int kTileElems = 4096;  // LDS: TQ (TP + 1) doubles, at most 33 KB

__global__ __launch_bounds__(256) void permute_tile_kernel(const double* __restrict__ in,
                                                           double* __restrict__ out, TDesc td) {
  extern __shared__ double tile[];  // TQ rows of TP + 1 (odd row stride: no bank pile-up)
  const long long tilesPQ = td.tilesP * td.tilesQ;
  const long long bidx = blockIdx.x / tilesPQ;
  const long long trem = blockIdx.x - bidx * tilesPQ;
  const long long tq = trem / td.tilesP;
  const long long tp = trem - tq * td.tilesP;
  long long rem = bidx, ioff = 0, ooff = 0;
  for (int a = td.nb - 1; a >= 0; --a) {
    const long long q = rem / td.bdim[a];
    const long long i = rem - q * td.bdim[a];
    ioff += i * td.bin[a];
    ooff += i * td.bout[a];
    rem = q;
  }
  const long long p0 = tp * td.TP, q0 = tq * td.TQ;
  // extents of this tile (the last tile along an axis may be partial); the
  // linear index runs over the np x nq elements only, so no thread idles on
  // a partial tile
  const int np = (int)min((long long)td.TP, td.dimP - p0);
  const int nq = (int)min((long long)td.TQ, td.dimQ - q0);
  const int ld = td.TP + 1;
  const int cnt = np * nq;
  // reads: runs of np consecutive P along each q
  for (int idx = threadIdx.x; idx < cnt; idx += 256) {
    const int q = idx / np, p = idx - q * np;
    tile[q * ld + p] = in[ioff + (q0 + q) * td.qs_in + p0 + p];
  }
  __syncthreads();
  // writes: runs of nq consecutive Q along each p
  for (int idx = threadIdx.x; idx < cnt; idx += 256) {
    const int p = idx / nq, q = idx - p * nq;
    out[ooff + (p0 + p) * td.ps_out + q0 + q] = tile[q * ld + p];
  }
}

}  // namespace

void permute(Context& ctx, const double* in, double* out, int rank, const long long* dims,
             const int* perm) {
  CTM_REQUIRE(rank >= 1 && rank <= 8, "permute: rank out of range");
  long long total = 1;
  long long istride[8];
  for (int a = rank - 1; a >= 0; --a) {
    istride[a] = total;
    total *= dims[a];
  }
  if (total == 0) return;
  // output dims and strides
  long long odim[8], istr_o[8], ostr[8];
  {
    long long s = 1;
    for (int a = rank - 1; a >= 0; --a) {
      odim[a] = dims[perm[a]];
      istr_o[a] = istride[perm[a]];
      ostr[a] = s;
      s *= odim[a];
    }
  }
  // merge consecutive output axes that are also consecutive in the input
  int r2 = 0;
  long long md[8], mi[8], mo[8];
  for (int a = 0; a < rank; ++a) {
    if (odim[a] == 1) continue;
    if (r2 > 0 && mi[r2 - 1] == istr_o[a] * odim[a]) {
      md[r2 - 1] *= odim[a];
      mi[r2 - 1] = istr_o[a];
      mo[r2 - 1] = ostr[a];
    } else {
      md[r2] = odim[a];
      mi[r2] = istr_o[a];
      mo[r2] = ostr[a];
      ++r2;
    }
  }
  if (r2 == 0) { md[0] = 1; mi[0] = 1; mo[0] = 1; r2 = 1; }
  const bool inner_kept = (mi[r2 - 1] == 1);
  if (inner_kept || r2 == 1) {
    PermDesc pd;
    pd.rank = r2;
    for (int a = 0; a < r2; ++a) { pd.odim[a] = md[a]; pd.istr[a] = mi[a]; pd.ostr[a] = mo[a]; }
    const int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(permute_copy_kernel, dim3(blocks), dim3(256), 0, ctx.stream, in, out, pd,
                       total);
    CTM_HIP(hipGetLastError());
    return;
  }
  // tiled transpose: Q = last output axis, P = the output axis with input stride 1
  int ap = -1;
  for (int a = 0; a < r2; ++a)
    if (mi[a] == 1) ap = a;
  CTM_REQUIRE(ap >= 0, "permute: no unit-stride axis");
  TDesc td;
  td.dimP = md[ap];
  td.dimQ = md[r2 - 1];
  td.qs_in = mi[r2 - 1];
  td.ps_out = mo[ap];
  td.nb = 0;
  for (int a = 0; a < r2 - 1; ++a) {
    if (a == ap) continue;
    td.bdim[td.nb] = md[a];
    td.bin[td.nb] = mi[a];
    td.bout[td.nb] = mo[a];
    ++td.nb;
  }
  // the whole plane along an axis when it is short, else 64 (P) or 32 (Q)
  td.TP = (int)(td.dimP <= 128 ? td.dimP : 64);
  td.TQ = (int)(td.dimQ <= 64 ? td.dimQ : 32);
  while ((long long)td.TP * td.TQ > kTileElems) td.TQ = (td.TQ + 1) / 2;
  td.tilesP = (td.dimP + td.TP - 1) / td.TP;
  td.tilesQ = (td.dimQ + td.TQ - 1) / td.TQ;
  long long batch = 1;
  for (int a = 0; a < td.nb; ++a) batch *= td.bdim[a];
  const long long blocks = batch * td.tilesP * td.tilesQ;
  CTM_REQUIRE(blocks < (1LL << 31), "permute: too many tiles");
  const size_t lds = (size_t)td.TQ * (td.TP + 1) * sizeof(double);
  hipLaunchKernelGGL(permute_tile_kernel, dim3((unsigned)blocks), dim3(256), lds, ctx.stream, in,
                     out, td);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
