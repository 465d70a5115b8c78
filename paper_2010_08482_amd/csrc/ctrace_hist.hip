// Histogram of a conserved sector label (Sec. 2.3.2, the impurity density-
// matrix estimator summed over the states of every label; Sec. 4.2, valence
// histogram).
//
// A projector P_l onto the sectors with label l commutes with H_loc and is
// the identity or zero on every sector, so inserting it at time tau keeps
// exactly the strings whose sector at tau carries label l, and its position
// inside an interval between two operators does not matter.  With w_s the
// weight of the string that starts in sector q0 (the same per-string values
// the combine kernels sum) and t_s(l) the time it spends in sectors of label
// l, the tau-integrated estimator of a configuration is
//
//     h_l = sum_s w_s t_s(l) / (beta * sum_s w_s).
//
// One workgroup per configuration, one thread per string; the string's
// interval lengths are summed per label while its sector walk is replayed
// (integer table lookups only), eight labels per pass.
#include <hip/hip_runtime.h>

#include "ctrace_internal.h"

namespace ctr {

namespace {

constexpr int kHistThreads = 256;
constexpr int kHistChunk = 8;  // labels per pass (register accumulators)

// Sum over the workgroup in a fixed order: wavefront butterflies, then the
// four wavefront partials in index order.
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(kHistThreads) void k_hist(DevImp I, BatchArgs B, HistArgs H) {
  __shared__ double s_dt[kMaxOps];
  __shared__ int s_op[kMaxOps];
  __shared__ double s_red[4];

  const int c = blockIdx.x;
  const int t = threadIdx.x;
  double* out = H.hist + (long long)c * H.n_labels * 2;
  const ctr_value v = B.out[c];
  const bool live = !(v.flags & (CTR_FLAG_INVALID | CTR_FLAG_REJECTED | CTR_FLAG_ZERO)) && (v.re != 0.0 || v.im != 0.0);
  if (!live) {
    for (int l = t; l < 2 * H.n_labels; l += kHistThreads) out[l] = 0.0;
    return;
  }
  const long long base = B.offsets[c];
  const int n = (int)(B.offsets[c + 1] - base);  // validated by the plan (live implies 0 <= n <= kMaxOps)
  for (int i = t; i < n; i += kHistThreads) {
    s_op[i] = B.op[base + i];
    s_dt[i] = i > 0 ? B.tau[base + i] - B.tau[base + i - 1] : B.tau[base] + I.beta - B.tau[base + n - 1];
  }
  __syncthreads();

  // string weights, on the scale of the combined value
  const double ln2 = 0.69314718055994530942;
  const double lm = v.log_scale + I.beta * I.E0;
  const StrRec* recs = B.rec + (long long)c * I.n_sec;
  double wr = 0.0, wi = 0.0;  // this thread's strings, summed
  for (int q0 = t; q0 < I.n_sec; q0 += kHistThreads) {
    const StrRec R = recs[q0];
    if (R.n_panels == 0) continue;
    const PanelRes* vals = H.colbase ? H.vals + H.colbase[B.cfg_off[c] + R.loc_off] : H.vals + B.cfg_off[c] + R.loc_off;
    const int nv = H.colbase ? R.width : R.n_panels;
    for (int j = 0; j < nv; ++j) {
      const PanelRes P = vals[j];
      if (P.re != 0.0 || P.im != 0.0) {
        const double f = exp(P.e2 * ln2 - R.L - lm);
        wr += P.re * f;
        wi += P.im * f;
      }
    }
  }
  const double Wr = block_sum(wr, s_red);
  const double Wi = block_sum(wi, s_red);
  // 1 / W = conj(W) / |W|^2, with W scaled to its larger component first
  const double Wm = fmax(fabs(Wr), fabs(Wi));
  if (!(Wm > 0.0)) {  // the string weights cancel exactly: no estimate
    for (int l = t; l < 2 * H.n_labels; l += kHistThreads) out[l] = 0.0;
    return;
  }
  const double ur = Wr / Wm, ui = Wi / Wm;
  const double den = (ur * ur + ui * ui) * Wm;

  for (int l0 = 0; l0 < H.n_labels; l0 += kHistChunk) {
    double ar[kHistChunk], ai[kHistChunk];
#pragma unroll
    for (int k = 0; k < kHistChunk; ++k) ar[k] = ai[k] = 0.0;
    for (int q0 = t; q0 < I.n_sec; q0 += kHistThreads) {
      const StrRec R = recs[q0];
      if (R.n_panels == 0) continue;
      // the string's weight again (same order as above)
      const PanelRes* vals = H.colbase ? H.vals + H.colbase[B.cfg_off[c] + R.loc_off] : H.vals + B.cfg_off[c] + R.loc_off;
      const int nv = H.colbase ? R.width : R.n_panels;
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < nv; ++j) {
        const PanelRes P = vals[j];
        if (P.re != 0.0 || P.im != 0.0) {
          const double f = exp(P.e2 * ln2 - R.L - lm);
          sr += P.re * f;
          si += P.im * f;
        }
      }
      // time in each label of the chunk along the string's sector walk; the
      // interval in front of operator p (the wrapped one for p = 0) is spent
      // in the sector the walk holds before p
      double tl[kHistChunk];
#pragma unroll
      for (int k = 0; k < kHistChunk; ++k) tl[k] = 0.0;
      int s = q0;
      if (n == 0) {
        const int lab = H.label[s] - l0;
#pragma unroll
        for (int k = 0; k < kHistChunk; ++k) tl[k] = lab == k ? I.beta : 0.0;
      }
      for (int p = 0; p < n; ++p) {
        const int lab = H.label[s] - l0;
        const double d = s_dt[p];
#pragma unroll
        for (int k = 0; k < kHistChunk; ++k) tl[k] += lab == k ? d : 0.0;
        s = I.next[s * I.nops + s_op[p]];  // a surviving string never reaches -1
      }
#pragma unroll
      for (int k = 0; k < kHistChunk; ++k) {
        ar[k] += sr * tl[k];
        ai[k] += si * tl[k];
      }
    }
#pragma unroll
    for (int k = 0; k < kHistChunk; ++k) {
      const double Ar = block_sum(ar[k], s_red) / I.beta;
      const double Ai = block_sum(ai[k], s_red) / I.beta;
      if (t == 0 && l0 + k < H.n_labels) {
        // (Ar + i Ai) / (Wr + i Wi)
        out[2 * (l0 + k)] = (Ar * ur + Ai * ui) / den;
        out[2 * (l0 + k) + 1] = (Ai * ur - Ar * ui) / den;
      }
    }
  }
}

}  // namespace

hipError_t launch_hist(const DevImp& imp, const BatchArgs& b, const HistArgs& h, hipStream_t stream) {
  if (b.n_cfg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hist, dim3(b.n_cfg), dim3(kHistThreads), 0, stream, imp, b, h);
  return hipGetLastError();
}

}  // namespace ctr
