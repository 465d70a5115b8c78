// gfx950 kernels of the CT-HYB local trace (block form of Sec. 3.3.1).
//
//   k_plan     one workgroup per configuration: validates the string, walks
//              the sector map s_alpha(q) for every start sector q0 (zero
//              sector = -1), rotates each surviving string to start at its
//              narrowest sector (trace cyclicity), accumulates the energy
//              shift and the lazy bound of Sec. 3.3.1, and scans panel counts.
//   k_scan     one workgroup: panel offsets of all configurations.
//   k_chain    persistent: one workgroup per (string, 16-column panel) pulls
//              work from an atomic counter and runs the whole chain
//              X <- F_op * P * X with X resident in LDS, the diagonal
//              propagator fused into the epilogue of the previous step, FP64
//              MFMA block products (16x16x4, or 4x4x4 on groups of four columns
//              for panels of at most 12 columns), and a per-column power-of-two
//              rescale from wavefront max-reductions; the last operator only
//              contributes the diagonal of F * X.
//   k_combine  one thread per configuration: merges the (mantissa, exponent)
//              panel results of all strings in a fixed order.
#include <math.h>

#include <algorithm>

#include "ctrace_internal.h"

namespace ctr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double dtp(const double* tau, int n, int p, double beta) {
  // imaginary-time gap in front of operator p; position 0 also carries the
  // gap after the last operator (the two end propagators merge by cyclicity)
  return p ? tau[p] - tau[p - 1] : tau[0] + beta - tau[n - 1];
}

// Lazy traces: a bound given by its log (without the -beta*E0 part), in
// integer units of 2^-kLazyUnitBits times the threshold exp(lthr), rounded up
// and capped at 2^kLazyCapBits (a capped panel alone exceeds the threshold,
// so the configuration cannot be rejected while it stays capped).
__device__ __forceinline__ unsigned long long lazy_units(double logb, double lthr) {
  const double ln2 = 0.69314718055994530942;
  const double x = logb - lthr + kLazyUnitBits * ln2;
  if (!(x < kLazyCapBits * ln2)) return 1ull << kLazyCapBits;  // also a NaN
  return (unsigned long long)ceil(exp(x) * (1.0 + 1e-12));
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPlanThreads) void k_plan(DevImp I, BatchArgs B) {
  __shared__ double s_tau[kMaxOps];
  __shared__ double s_dt[kMaxOps];
  __shared__ int s_op[kMaxOps];
  __shared__ int s_bad;
  __shared__ int s_scan[kPlanThreads];
  __shared__ double s_red[kPlanThreads];
  __shared__ unsigned long long s_units[kPlanThreads];

  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const long long base = B.offsets[c];
  const long long nl = B.offsets[c + 1] - base;
  if (t == 0) s_bad = (nl < 0 || nl > kMaxOps) ? 1 : 0;
  __syncthreads();
  const int n = s_bad ? 0 : (int)nl;
  for (int i = t; i < n; i += kPlanThreads) {
    s_tau[i] = B.tau[base + i];
    s_op[i] = B.op[base + i];
  }
  __syncthreads();
  int bad = 0;
  for (int i = t; i < n; i += kPlanThreads) {
    const double x = s_tau[i];
    const int o = s_op[i];
    if (!(x >= 0.0 && x < I.beta)) bad = 1;
    if (o < 0 || o >= I.nops) bad = 1;
    if (i > 0 && !(x >= s_tau[i - 1])) bad = 1;
    s_dt[i] = (i > 0) ? x - s_tau[i - 1] : x + I.beta - s_tau[n - 1];
  }
  if (bad) atomicOr(&s_bad, 1);
  __syncthreads();
  bad = s_bad;

  const int chunk = (I.n_sec + kPlanThreads - 1) / kPlanThreads;
  const int q_lo = min(t * chunk, I.n_sec);
  const int q_hi = min(q_lo + chunk, I.n_sec);
  StrRec* recs = B.rec + (long long)c * I.n_sec;
  int my_panels = 0, my_nstr = 0;
  unsigned long long my_units = 0;
  double my_max = -INFINITY;
  for (int q0 = q_lo; q0 < q_hi; ++q0) {
    StrRec R;
    R.q_start = q0;
    R.jstar = 0;
    R.width = I.dim[q0];
    R.n_panels = 0;
    R.loc_off = 0;
    R.pad = 0;
    R.L = 0.0;
    R.logB = -INFINITY;
    R.u_full = R.u_last = 0;
    if (!bad) {
      int s = q0, best = I.dim[q0], jstar = 0, qbest = q0;
      double L = 0.0, logn = 0.0;
      bool alive = true;
      for (int p = 0; p < n; ++p) {
        const int d = I.dim[s];
        if (d < best) {
          best = d;
          jstar = p;
          qbest = s;
        }
        L += s_dt[p] * (I.emin[s] - I.E0);
        const int idx = s * I.nops + s_op[p];
        logn += I.lognorm[idx];
        s = I.next[idx];
        if (s < 0) {
          alive = false;
          break;
        }
      }
      if (alive && s == q0) {
        if (n == 0) L = I.beta * (I.emin[q0] - I.E0);
        R.q_start = qbest;
        R.jstar = jstar;
        R.width = best;
        R.n_panels = (best + B.panel - 1) / B.panel;
        R.L = L;
        R.logB = log((double)best) - L + logn;
        if (B.log_thr != nullptr) {
          // initial panel bounds: ncols * exp(-L) * (block norms), ncols = panel width or the remainder
          const double lthr = B.log_thr[c] + I.beta * I.E0;
          const int last = best - (R.n_panels - 1) * B.panel;
          R.u_full = lazy_units(log((double)B.panel) - L + logn, lthr);
          R.u_last = lazy_units(log((double)last) - L + logn, lthr);
          my_units += (unsigned long long)(R.n_panels - 1) * R.u_full + R.u_last;
        }
        my_panels += R.n_panels;
        my_nstr += 1;
        my_max = fmax(my_max, R.logB);
      }
    }
    recs[q0] = R;
  }

  // panel offsets inside the configuration (inclusive scan of the chunks)
  s_scan[t] = my_panels;
  __syncthreads();
  for (int off = 1; off < kPlanThreads; off <<= 1) {
    const int v = (t >= off) ? s_scan[t - off] : 0;
    __syncthreads();
    s_scan[t] += v;
    __syncthreads();
  }
  const int total = s_scan[kPlanThreads - 1];
  int run = s_scan[t] - my_panels;
  for (int q0 = q_lo; q0 < q_hi; ++q0) {
    recs[q0].loc_off = run;
    run += recs[q0].n_panels;
  }
  __syncthreads();

  // log of the summed bound: max, then sum of exp(logB - max), fixed order
  s_red[t] = my_max;
  __syncthreads();
  for (int off = kPlanThreads / 2; off > 0; off >>= 1) {
    if (t < off) s_red[t] = fmax(s_red[t], s_red[t + off]);
    __syncthreads();
  }
  const double gmax = s_red[0];
  __syncthreads();
  double my_sum = 0.0;
  if (gmax > -INFINITY)
    for (int q0 = q_lo; q0 < q_hi; ++q0)
      if (recs[q0].n_panels > 0) my_sum += exp(recs[q0].logB - gmax);
  s_red[t] = my_sum;
  s_scan[t] = my_nstr;
  s_units[t] = my_units;
  __syncthreads();
  for (int off = kPlanThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_red[t] += s_red[t + off];
      s_scan[t] += s_scan[t + off];
      s_units[t] += s_units[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int nstr = s_scan[0];
    const double logB = nstr > 0 ? gmax + log(s_red[0]) - I.beta * I.E0 : -INFINITY;
    int flags = bad ? CTR_FLAG_INVALID : 0;
    int cnt = bad ? 0 : total;
    if (!bad && nstr == 0) flags |= CTR_FLAG_ZERO;
    B.cfg_rej[c] = 0;
    if (B.log_thr != nullptr) {
      B.cfg_lthr[c] = B.log_thr[c] + I.beta * I.E0;
      B.cfg_bsum[c] = s_units[0];
      if (!bad && nstr > 0 && logB < B.log_thr[c]) {
        flags |= CTR_FLAG_REJECTED;
        cnt = 0;
      }
    }
    B.cfg_cnt[c] = cnt;
    B.cfg_flags[c] = flags;
    B.cfg_nstr[c] = bad ? 0 : nstr;
    B.cfg_logB[c] = bad ? -INFINITY : logB;
  }
}

// ---------------------------------------------------------------------------
// scan of per-configuration panel counts
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_scan(BatchArgs B) {
  __shared__ long long s[1024];
  const int t = threadIdx.x;
  const int n = B.n_cfg;
  const int chunk = (n + 1023) / 1024;
  const int lo = min(t * chunk, n);
  const int hi = min(lo + chunk, n);
  long long sum = 0;
  for (int i = lo; i < hi; ++i) sum += B.cfg_cnt[i];
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long v = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  long long run = s[t] - sum;
  for (int i = lo; i < hi; ++i) {
    B.cfg_off[i] = run;
    run += B.cfg_cnt[i];
  }
  if (t == 1023) B.cfg_off[n] = s[1023];
  if (t == 0) *B.counter = 0u;
}

// ---------------------------------------------------------------------------
// chain
// ---------------------------------------------------------------------------
template <bool CPLX, int NW>
__host__ __device__ constexpr size_t chain_lds_bytes_t(int xr, int n_sec, int next_entries) {
  return 8 * ((size_t)(CPLX ? 2 : 1) * xr * kPanel + 2 * (size_t)xr + NW * kPanel + (CPLX ? 2 : 1) * NW * 64 +
              kMaxOps) +
         4 * (kPanel + 2 * (size_t)n_sec) + 2 * (2 * (size_t)kMaxOps + 2 + next_entries);
}

// Lazy traces: every panel starts with its share of the string bound,
// ncols * exp(-L) times the block norms, and replaces it while its chain runs
// by sqrt(ncols) * ||X||_F * exp(-L) (the sum of ncols diagonal entries of
// R * X is at most sqrt(ncols) ||R X||_F, and the remaining blocks and shifted
// propagators R have norm <= 1), and at its end by the modulus of its exact
// contribution.  The configuration's running sum (integer threshold units)
// only decreases; once it is below the threshold the configuration is
// rejected and its remaining panels stop.
__device__ __forceinline__ bool lazy_rejected(const BatchArgs& B, int c) {
  return __hip_atomic_load(B.cfg_rej + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ unsigned long long lazy_initial(const StrRec& R, int local) {
  return (local - R.loc_off == R.n_panels - 1) ? R.u_last : R.u_full;
}

// Replaces the panel's bound *ucur by the bound with log logb if that is
// smaller; returns true if the configuration is now rejected.
__device__ __forceinline__ bool lazy_update(const BatchArgs& B, int c, unsigned long long* ucur, double logb) {
  const unsigned long long unew = lazy_units(logb, B.cfg_lthr[c]);
  if (unew >= *ucur) return false;
  const unsigned long long delta = unew - *ucur;  // two's complement: subtracts
  *ucur = unew;
  const unsigned long long sum = atomicAdd(B.cfg_bsum + c, delta) + delta;
  if (sum < (1ull << kLazyUnitBits)) {
    atomicExch(B.cfg_rej + c, 1);
    return true;
  }
  return false;
}

// log of sum_j exp(a_j) over the 4 lanes of a quad-aligned group (xor 1, 2)
__device__ __forceinline__ double logsumexp_quad(double a) {
  double m = a;
  m = fmax(m, __shfl_xor(m, 1));
  m = fmax(m, __shfl_xor(m, 2));
  double e = (m == -INFINITY) ? 0.0 : exp(a - m);
  e += __shfl_xor(e, 1);
  e += __shfl_xor(e, 2);
  return (m == -INFINITY) ? -INFINITY : m + log(e);
}

// One chain step for a panel of at most 12 columns: FP64 MFMA 4x4x4 with four
// blocks stacked along the rows, so a 16-row tile times a group of 4 columns
// is one instruction and only ceil(ncols/4) column groups are computed.
// Lane l holds A[row l%16][k l/16] (as for 16x16x4), B[k l/16][col l%4] and
// D[row 4*((l%16)/4) + l/16][col l%4].
template <bool CPLX, int NW, int MAXT>
__device__ __forceinline__ void step_narrow(int t, const double* __restrict__ Fr, const double* __restrict__ Fi,
                                            int ld, int ntiles, int d_in, const double* pa, const double* pb,
                                            double* Xr, double* Xi, double* cmax, int* colexp, int col0,
                                            int ncols, int G, int lane, int wave, int tid) {
  const int ln = lane & 15, lq = lane >> 4, l3 = lane & 3;
  const int orow = 4 * (ln >> 2) + lq;
  double acc_r[MAXT][3], acc_i[MAXT][3];
#pragma unroll
  for (int tt = 0; tt < MAXT; ++tt)
#pragma unroll
    for (int g = 0; g < 3; ++g) acc_r[tt][g] = acc_i[tt][g] = 0.0;
  if (t == 0) {
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
      const int tile = wave + tt * NW;
      if (tile < ntiles) {
#pragma unroll
        for (int g = 0; g < 3; ++g) {
          const int c = g * 4 + l3;
          if (g < G && c < ncols) {
            const int k = col0 + c;
            const long long a = (long long)k * ld + tile * 16 + orow;
            const double p = pa[k];
            acc_r[tt][g] = Fr[a] * p;
            if (CPLX) acc_i[tt][g] = Fi[a] * p;
          }
        }
      }
    }
  } else {
    const int ksteps = (d_in + 3) >> 2;
    for (int kc = 0; kc < ksteps; ++kc) {
      const int krow = kc * 4 + lq;
      double br[3], bi[3];
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        br[g] = (g < G) ? Xr[krow * kPanel + g * 4 + l3] : 0.0;
        bi[g] = (CPLX && g < G) ? Xi[krow * kPanel + g * 4 + l3] : 0.0;
      }
#pragma unroll
      for (int tt = 0; tt < MAXT; ++tt) {
        const int tile = wave + tt * NW;
        if (tile < ntiles) {
          const long long a = (long long)krow * ld + tile * 16 + ln;
          const double ar = Fr[a];
          const double ai = CPLX ? Fi[a] : 0.0;
#pragma unroll
          for (int g = 0; g < 3; ++g) {
            if (g < G) {
              acc_r[tt][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar, br[g], acc_r[tt][g], 0, 0, 0);
              if (CPLX) {
                acc_r[tt][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(-ai, bi[g], acc_r[tt][g], 0, 0, 0);
                acc_i[tt][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar, bi[g], acc_i[tt][g], 0, 0, 0);
                acc_i[tt][g] = __builtin_amdgcn_mfma_f64_4x4x4f64(ai, br[g], acc_i[tt][g], 0, 0, 0);
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();  // X consumed by every wave; pb complete

  double cm[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int tt = 0; tt < MAXT; ++tt) {
    const int tile = wave + tt * NW;
    if (tile < ntiles) {
      const double p = pb[tile * 16 + orow];
#pragma unroll
      for (int g = 0; g < 3; ++g) {
        acc_r[tt][g] *= p;
        cm[g] = fmax(cm[g], fabs(acc_r[tt][g]));
        if (CPLX) {
          acc_i[tt][g] *= p;
          cm[g] = fmax(cm[g], fabs(acc_i[tt][g]));
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    cm[g] = fmax(cm[g], __shfl_xor(cm[g], 4));
    cm[g] = fmax(cm[g], __shfl_xor(cm[g], 8));
    cm[g] = fmax(cm[g], __shfl_xor(cm[g], 16));
    cm[g] = fmax(cm[g], __shfl_xor(cm[g], 32));
  }
  if (lane < 4) {
#pragma unroll
    for (int g = 0; g < 3; ++g)
      if (g < G) cmax[wave * kPanel + g * 4 + lane] = cm[g];
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    if (g < G) {
      double M = 0.0;
#pragma unroll
      for (int w2 = 0; w2 < NW; ++w2) M = fmax(M, cmax[w2 * kPanel + g * 4 + l3]);
      int e = 0;
      if (M > 0.0) frexp(M, &e);
      const double sc = ldexp(1.0, -e);
      if (tid < 4) colexp[g * 4 + tid] += e;
#pragma unroll
      for (int tt = 0; tt < MAXT; ++tt) {
        const int tile = wave + tt * NW;
        if (tile < ntiles) {
          const int m = tile * 16 + orow;
          Xr[m * kPanel + g * 4 + l3] = acc_r[tt][g] * sc;
          if (CPLX) Xi[m * kPanel + g * 4 + l3] = acc_i[tt][g] * sc;
        }
      }
    }
  }
  __syncthreads();
}

// One chain step in FP32-split precision.  Every operand is cut into
// NSL (6 or 7) integer-valued slices of kSliceBits bits (F per row, scaled by the
// row's power of two; X per column, already in (-1, 1) after the rescale):
//   f = sum_s A_s 2^{-b s},  x = sum_t B_t 2^{-b t},  |A_s|, |B_t| < 2^b.
// The products A_s B_t with s + t <= NSL + 1 run on FP32 MFMA 16x16x4.
// Slice products are integers below 2^{2b}; with at most NSL products per
// level and split_chunk() values of k per chunk, every partial sum stays below
// 2^24, so the FP32 accumulation is exact.  After each chunk the level sums
// are converted to FP64 (exact) and added with their weights 2^{-b L}; the
// eigenvalue propagators, the rescale and the final trace stay FP64.
constexpr int kSliceBits = 8;
// values of k per exact chunk: 6 slices 40 real / 20 complex, 7 slices 36 / 16
// (a complex level sum takes two products per slice pair)
template <bool CPLX, int NSL>
__host__ __device__ constexpr int split_chunk() {
  return ((1 << (24 - 2 * kSliceBits)) / (NSL * (CPLX ? 2 : 1))) & ~3;
}

// D layout of the FP32 16x16x4 MFMA: item i of lane l is row f32_row(i, l/16), column l%16.
__device__ __forceinline__ int f32_row(int i, int lq) { return 4 * lq + i; }

template <int NSL>
__device__ __forceinline__ void slice_digits(double v, float* d) {
#pragma unroll
  for (int s = 0; s < NSL; ++s) {
    v *= (double)(1 << kSliceBits);
    const double a = trunc(v);
    d[s] = (float)a;
    v -= a;
  }
}

template <bool CPLX, int NW, int MAXT, int NSL>
__device__ __forceinline__ void step_split(int t, const double* __restrict__ Fr, const double* __restrict__ Fi,
                                           const short* __restrict__ rexp, int ld, int ntiles, int d_in,
                                           const double* pa, const double* pb, double* Xr, double* Xi,
                                           double* cmax, int* colexp, int col0, int ncols, int lane, int wave,
                                           int tid) {
  typedef float flt4 __attribute__((ext_vector_type(4)));
  const int ln = lane & 15, lq = lane >> 4;
  double acc_r[MAXT][4], acc_i[MAXT][4];
#pragma unroll
  for (int tt = 0; tt < MAXT; ++tt)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc_r[tt][i] = acc_i[tt][i] = 0.0;

  if (t == 0) {
    // column-scaled copy of F (no product), already in the FP32 D layout
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
      const int tile = wave + tt * NW;
      if (tile < ntiles && ln < ncols) {
        const int k = col0 + ln;
        const double p = pa[k];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const long long a = (long long)k * ld + tile * 16 + f32_row(i, lq);
          acc_r[tt][i] = Fr[a] * p;
          if (CPLX) acc_i[tt][i] = Fi[a] * p;
        }
      }
    }
  } else {
    // inverse row scale of the A rows this lane feeds (row tile*16 + ln)
    double ainv[MAXT];
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
      const int tile = wave + tt * NW;
      ainv[tt] = (tile < ntiles) ? ldexp(1.0, -(int)rexp[tile * 16 + ln]) : 0.0;
    }
    const int ksteps = (d_in + 3) >> 2;
    for (int k0 = 0; k0 < ksteps; k0 += split_chunk<CPLX, NSL>() / 4) {
      const int k1 = min(ksteps, k0 + split_chunk<CPLX, NSL>() / 4);
      flt4 lr[MAXT][NSL], li[MAXT][NSL];
#pragma unroll
      for (int tt = 0; tt < MAXT; ++tt)
#pragma unroll
        for (int L = 0; L < NSL; ++L) {
          lr[tt][L] = flt4{0.f, 0.f, 0.f, 0.f};
          li[tt][L] = flt4{0.f, 0.f, 0.f, 0.f};
        }
      for (int kc = k0; kc < k1; ++kc) {
        const int krow = kc * 4 + lq;
        float bxr[NSL], bxi[NSL];
        slice_digits<NSL>(Xr[krow * kPanel + ln], bxr);
        if (CPLX) slice_digits<NSL>(Xi[krow * kPanel + ln], bxi);
#pragma unroll
        for (int tt = 0; tt < MAXT; ++tt) {
          const int tile = wave + tt * NW;
          if (tile < ntiles) {
            const long long a = (long long)krow * ld + tile * 16 + ln;
            float afr[NSL], afi[NSL], afn[NSL];
            slice_digits<NSL>(Fr[a] * ainv[tt], afr);
            if (CPLX) {
              slice_digits<NSL>(Fi[a] * ainv[tt], afi);
#pragma unroll
              for (int s2 = 0; s2 < NSL; ++s2) afn[s2] = -afi[s2];
            }
            // level L = s + t (slice indices from 1), kept for L <= NSL + 1
#pragma unroll
            for (int L = 2; L <= NSL + 1; ++L) {
#pragma unroll
              for (int s1 = 1; s1 < L; ++s1) {
                const int t1 = L - s1;
                lr[tt][L - 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[s1 - 1], bxr[t1 - 1], lr[tt][L - 2], 0, 0, 0);
                if (CPLX) {
                  lr[tt][L - 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(afn[s1 - 1], bxi[t1 - 1], lr[tt][L - 2], 0, 0, 0);
                  li[tt][L - 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[s1 - 1], bxi[t1 - 1], li[tt][L - 2], 0, 0, 0);
                  li[tt][L - 2] = __builtin_amdgcn_mfma_f32_16x16x4f32(afi[s1 - 1], bxr[t1 - 1], li[tt][L - 2], 0, 0, 0);
                }
              }
            }
          }
        }
      }
      // exact FP32 level sums -> FP64 with weights 2^{-b L}
#pragma unroll
      for (int tt = 0; tt < MAXT; ++tt) {
#pragma unroll
        for (int L = 2; L <= NSL + 1; ++L) {
          const double wgt = ldexp(1.0, -kSliceBits * L);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            acc_r[tt][i] += (double)lr[tt][L - 2][i] * wgt;
            if (CPLX) acc_i[tt][i] += (double)li[tt][L - 2][i] * wgt;
          }
        }
      }
    }
    // undo the row scales of the output rows
#pragma unroll
    for (int tt = 0; tt < MAXT; ++tt) {
      const int tile = wave + tt * NW;
      if (tile < ntiles) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double f = ldexp(1.0, (int)rexp[tile * 16 + f32_row(i, lq)]);
          acc_r[tt][i] *= f;
          acc_i[tt][i] *= f;
        }
      }
    }
  }
  __syncthreads();  // X consumed by every wave; pb complete

  double cm = 0.0;
#pragma unroll
  for (int tt = 0; tt < MAXT; ++tt) {
    const int tile = wave + tt * NW;
    if (tile < ntiles) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double p = pb[tile * 16 + f32_row(i, lq)];
        acc_r[tt][i] *= p;
        cm = fmax(cm, fabs(acc_r[tt][i]));
        if (CPLX) {
          acc_i[tt][i] *= p;
          cm = fmax(cm, fabs(acc_i[tt][i]));
        }
      }
    }
  }
  cm = fmax(cm, __shfl_xor(cm, 16));
  cm = fmax(cm, __shfl_xor(cm, 32));
  if (lane < 16) cmax[wave * kPanel + lane] = cm;
  __syncthreads();
  double M = 0.0;
#pragma unroll
  for (int w2 = 0; w2 < NW; ++w2) M = fmax(M, cmax[w2 * kPanel + ln]);
  int e = 0;
  if (M > 0.0) frexp(M, &e);
  const double sc = ldexp(1.0, -e);
  if (tid < kPanel) colexp[tid] += e;
#pragma unroll
  for (int tt = 0; tt < MAXT; ++tt) {
    const int tile = wave + tt * NW;
    if (tile < ntiles) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = tile * 16 + f32_row(i, lq);
        Xr[m * kPanel + ln] = acc_r[tt][i] * sc;
        if (CPLX) Xi[m * kPanel + ln] = acc_i[tt][i] * sc;
      }
    }
  }
  __syncthreads();
}

template <bool CPLX, int NW, int MAXT, int SPLIT>
__global__ __launch_bounds__(NW * 64) void k_chain(DevImp I, BatchArgs B) {
  extern __shared__ double lds[];
  constexpr int NT = NW * 64;
  const int XR = I.xrows;
  const int NS = I.n_sec;
  double* Xr = lds;                                    // [XR][16]
  double* Xi = lds + XR * kPanel;                      // [XR][16], complex only
  double* pa = lds + (CPLX ? 2 : 1) * XR * kPanel;     // propagator at the start position
  double* pb = pa + XR;                                // propagator in front of the next operator
  double* cmax = pb + XR;                              // [NW][16]
  double* red = cmax + NW * kPanel;                    // [NT] (x2 complex)
  double* s_dt = red + (CPLX ? 2 : 1) * NT;            // [kMaxOps] gap in front of every position
  int* colexp = (int*)(s_dt + kMaxOps);                // [16] per-column power of two
  int* s_dim = colexp + kPanel;                        // [NS] sector dimensions
  int* s_eoff = s_dim + NS;                            // [NS] energy offsets
  short* s_op = (short*)(s_eoff + NS);                 // [kMaxOps] operator codes, rotated order
  short* s_path = s_op + kMaxOps;                      // [kMaxOps + 1] sector before every step
  short* s_next = s_path + kMaxOps + 2;                // [NS * nops] sector map, when it fits
  __shared__ long long s_w;
  __shared__ int s_rej;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ln = lane & 15;  // column of the 16x16 tile held by this lane
  const int lq = lane >> 4;  // row group: D item i of this lane is row 4*i + lq
  const long long total = B.cfg_off[B.n_cfg];
  const bool next_in_lds = I.next_lds != 0;

  // per-impurity tables staged once for the lifetime of the workgroup
  for (int i = tid; i < NS; i += NT) {
    s_dim[i] = I.dim[i];
    s_eoff[i] = I.eoff[i];
  }
  if (next_in_lds)
    for (int i = tid; i < NS * I.nops; i += NT) s_next[i] = (short)I.next[i];

  for (;;) {
    if (tid == 0) s_w = (long long)atomicAdd(B.counter, 1u);
    __syncthreads();
    const long long w = s_w;
    if (w >= total) break;

    // locate (configuration, string, panel) of work item w
    int lo = 0, hi = B.n_cfg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.cfg_off[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const int local = (int)(w - B.cfg_off[c]);
    const StrRec* recs = B.rec + (long long)c * NS;
    lo = 0;
    hi = NS - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
    }
    const StrRec R = recs[lo];
    const int col0 = (local - R.loc_off) * kPanel;
    const int ncols = min(kPanel, R.width - col0);
    const int G = (ncols + 3) >> 2;     // groups of 4 columns
    const bool narrow = G <= 3;
    const long long base = B.offsets[c];
    const int n = (int)(B.offsets[c + 1] - base);

    // the string in LDS: operator codes and gaps in rotated order, then the
    // sectors it visits (one thread walks the sector map)
    for (int t = tid; t < n; t += NT) {
      const int p = (R.jstar + t) % n;
      s_op[t] = (short)B.op[base + p];
      s_dt[t] = p ? B.tau[base + p] - B.tau[base + p - 1] : B.tau[base] + I.beta - B.tau[base + n - 1];
    }
    if (tid < kPanel) colexp[tid] = 0;
    __syncthreads();
    if (tid == 0) {
      int q = R.q_start;
      s_path[0] = (short)q;
      if (next_in_lds) {
        for (int t = 0; t < n; ++t) {
          q = s_next[q * I.nops + s_op[t]];
          s_path[t + 1] = (short)q;
        }
      } else {
        for (int t = 0; t < n; ++t) {
          q = I.next[q * I.nops + s_op[t]];
          s_path[t + 1] = (short)q;
        }
      }
    }
    {
      const int s0 = R.q_start;
      const int d = s_dim[s0];
      const double dt = (n == 0) ? I.beta : s_dt[0];
      const double* e = I.esh + s_eoff[s0];
      for (int r = tid; r < XR; r += NT) pa[r] = (r < d) ? exp(-dt * e[r]) : 0.0;
    }
    __syncthreads();

    PanelRes out;
    out.re = out.im = out.e2 = 0.0;
    const bool lazy = B.log_thr != nullptr;
    unsigned long long ucur = lazy ? lazy_initial(R, local) : 0;  // used by thread 0
    bool dead = false;
    if (n == 0) {
      if (tid == 0) {
        double sum = 0.0;
        for (int cc = 0; cc < ncols; ++cc) sum += pa[col0 + cc];
        out.re = sum;
      }
    } else {
      long long boff_next = I.boff[s_path[0] * I.nops + s_op[0]];
      long long roff_next = SPLIT ? I.roff[s_path[0] * I.nops + s_op[0]] : 0;
      for (int t = 0; t < n - 1; ++t) {
        if (lazy) {
          if (tid == 0) s_rej = lazy_rejected(B, c) ? 1 : 0;
          __syncthreads();
          if (s_rej) {
            dead = true;
            break;
          }
        }
        const long long roff_cur = roff_next;
        const int s = s_path[t], s2 = s_path[t + 1];
        const int d_in = s_dim[s], d_out = s_dim[s2];
        const int ld = (d_out + 15) & ~15;
        const int ntiles = ld >> 4;
        const double* Fr = I.pool + boff_next;
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        // block of the next step: its address is known from the path, load it now
        boff_next = I.boff[s2 * I.nops + s_op[t + 1]];
        if (SPLIT) roff_next = I.roff[s2 * I.nops + s_op[t + 1]];
        {
          const double dt2 = s_dt[t + 1];
          const double* e = I.esh + s_eoff[s2];
          for (int r = tid; r < ld; r += NT) pb[r] = (r < d_out) ? exp(-dt2 * e[r]) : 0.0;
        }
        if (SPLIT) {
          step_split<CPLX, NW, MAXT, (SPLIT > 0 ? SPLIT : 6)>(t, Fr, Fi, I.rexp + roff_cur, ld, ntiles, d_in, pa, pb, Xr, Xi, cmax, colexp,
                                     col0, ncols, lane, wave, tid);
          continue;
        }
        if (narrow) {
          step_narrow<CPLX, NW, MAXT>(t, Fr, Fi, ld, ntiles, d_in, pa, pb, Xr, Xi, cmax, colexp, col0, ncols,
                                      G, lane, wave, tid);
          continue;
        }
        dbl4 acc_r[MAXT], acc_i[MAXT];
#pragma unroll
        for (int tt = 0; tt < MAXT; ++tt) {
          acc_r[tt] = dbl4{0.0, 0.0, 0.0, 0.0};
          acc_i[tt] = dbl4{0.0, 0.0, 0.0, 0.0};
        }
        if (t == 0) {
          // X is the identity on the panel columns times the start propagator:
          // F * X is a column-scaled copy of F.
          const int k = col0 + ln;
#pragma unroll
          for (int tt = 0; tt < MAXT; ++tt) {
            const int tile = wave + tt * NW;
            if (tile < ntiles && ln < ncols) {
              const double p = pa[k];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const long long a = (long long)k * ld + tile * 16 + 4 * i + lq;
                acc_r[tt][i] = Fr[a] * p;
                if (CPLX) acc_i[tt][i] = Fi[a] * p;
              }
            }
          }
        } else {
          const int ksteps = (d_in + 3) >> 2;
#pragma unroll 2
          for (int kc = 0; kc < ksteps; ++kc) {
            const int krow = kc * 4 + lq;
            const double br = Xr[krow * kPanel + ln];
            const double bi = CPLX ? Xi[krow * kPanel + ln] : 0.0;
#pragma unroll
            for (int tt = 0; tt < MAXT; ++tt) {
              const int tile = wave + tt * NW;
              if (tile < ntiles) {
                const long long a = (long long)krow * ld + tile * 16 + ln;
                const double ar = Fr[a];
                acc_r[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, acc_r[tt], 0, 0, 0);
                if (CPLX) {
                  const double ai = Fi[a];
                  acc_r[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, acc_r[tt], 0, 0, 0);
                  acc_i[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acc_i[tt], 0, 0, 0);
                  acc_i[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acc_i[tt], 0, 0, 0);
                }
              }
            }
          }
        }
        __syncthreads();  // X consumed by every wave; pb complete

        // fused propagator of the next position, then per-column max
        double cm = 0.0;
#pragma unroll
        for (int tt = 0; tt < MAXT; ++tt) {
          const int tile = wave + tt * NW;
          if (tile < ntiles) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double p = pb[tile * 16 + 4 * i + lq];
              acc_r[tt][i] *= p;
              cm = fmax(cm, fabs(acc_r[tt][i]));
              if (CPLX) {
                acc_i[tt][i] *= p;
                cm = fmax(cm, fabs(acc_i[tt][i]));
              }
            }
          }
        }
        cm = fmax(cm, __shfl_xor(cm, 16));
        cm = fmax(cm, __shfl_xor(cm, 32));
        if (lane < 16) cmax[wave * kPanel + lane] = cm;
        __syncthreads();
        double M = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < NW; ++w2) M = fmax(M, cmax[w2 * kPanel + ln]);
        int e = 0;
        if (M > 0.0) frexp(M, &e);
        const double sc = ldexp(1.0, -e);
        if (tid < kPanel) colexp[tid] += e;
#pragma unroll
        for (int tt = 0; tt < MAXT; ++tt) {
          const int tile = wave + tt * NW;
          if (tile < ntiles) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m = tile * 16 + 4 * i + lq;
              Xr[m * kPanel + ln] = acc_r[tt][i] * sc;
              if (CPLX) Xi[m * kPanel + ln] = acc_i[tt][i] * sc;
            }
          }
        }
        __syncthreads();
      }

      // last operator: only the diagonal of F * X (rows col0 .. col0+ncols)
      if (!dead) {
        const int s = s_path[n - 1];
        const int d_in = s_dim[s];
        const int ld = (s_dim[s_path[n]] + 15) & ~15;
        const double* Fr = I.pool + boff_next;
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        const int cc = tid & 15;
        double sr = 0.0, si = 0.0;
        if (cc < ncols) {
          for (int k = tid >> 4; k < d_in; k += NT / 16) {
            const long long a = (long long)k * ld + col0 + cc;
            const double fr = Fr[a], xr = Xr[k * kPanel + cc];
            if (CPLX) {
              const double fi = Fi[a], xi = Xi[k * kPanel + cc];
              sr += fr * xr - fi * xi;
              si += fr * xi + fi * xr;
            } else {
              sr += fr * xr;
            }
          }
        }
        red[tid] = sr;
        if (CPLX) red[NT + tid] = si;
        __syncthreads();
        if (tid < kPanel) {
          double vr = 0.0, vi = 0.0;
          for (int j = 0; j < NT / 16; ++j) {
            vr += red[j * 16 + tid];
            if (CPLX) vi += red[NT + j * 16 + tid];
          }
          cmax[tid] = vr;
          cmax[kPanel + tid] = vi;
        }
        __syncthreads();
        if (tid == 0) {
          int emax = INT_MIN;
          for (int j = 0; j < ncols; ++j)
            if (cmax[j] != 0.0 || cmax[kPanel + j] != 0.0) emax = max(emax, colexp[j]);
          if (emax != INT_MIN) {
            double vr = 0.0, vi = 0.0;
            for (int j = 0; j < ncols; ++j) {
              const double f = ldexp(1.0, colexp[j] - emax);
              vr += cmax[j] * f;
              vi += cmax[kPanel + j] * f;
            }
            out.re = vr;
            out.im = vi;
            out.e2 = (double)emax;
          }
          if (lazy) {
            const double a = hypot(out.re, out.im);
            lazy_update(B, c, &ucur, a > 0.0 ? log(a) + out.e2 * 0.69314718055994530942 - R.L : -INFINITY);
          }
        }
      }
    }
    if (tid == 0) B.res[w] = out;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// chain, one wavefront per panel (sectors of at most 128 states)
// ---------------------------------------------------------------------------
// Every wavefront of the workgroup pulls its own work item (a panel of at most
// kWavePanel columns) and runs the whole chain alone: all row tiles of the
// block product are in its registers, so the per-column max is a wavefront
// reduction and the step loop has no workgroup barrier.  Block products use
// FP64 MFMA 4x4x4 on groups of four columns: lane l holds A[row l%16][k l/16],
// B[k l/16][col l%4] and D[row 4*((l%16)/4) + l/16][col l%4].
constexpr int kWavePanel = 8;
constexpr int kWaveTiles = 8;  // 16-row tiles per wavefront: sectors up to 128 states
constexpr int kTileBatch = 4;  // nonzero k-steps of one row tile loaded together

template <bool CPLX>
__host__ __device__ constexpr size_t wave_region_bytes(int xr) {
  return (8 * ((size_t)(CPLX ? 2 : 1) * xr * kWavePanel + xr) + kMaxOps + 2 * ((size_t)kMaxOps + 2) + 15) & ~(size_t)15;
}

template <bool CPLX>
__host__ __device__ constexpr size_t wave_lds_bytes(int xr, int n_sec, int next_entries) {
  // per wavefront: X (kWavePanel columns, x2 complex), propagator, operator codes, path
  return 4 * wave_region_bytes<CPLX>(xr) + 4 * 2 * (size_t)n_sec + 2 * (size_t)next_entries + 64;
}

template <bool CPLX, bool LAZY>
__global__ __launch_bounds__(256, CPLX ? 2 : (LAZY ? 3 : 4)) void k_chain_wave(DevImp I, BatchArgs B) {
  extern __shared__ double lds[];
  const int XR = I.xrows;
  const int NS = I.n_sec;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ln = lane & 15, lq = lane >> 4, l3 = lane & 3;
  const int orow = 4 * (ln >> 2) + lq;  // D row of this lane inside a 16-row tile

  // per-wavefront region
  const size_t per_wave = wave_region_bytes<CPLX>(XR);
  char* my = (char*)lds + wave * per_wave;
  double* Xr = (double*)my;
  double* Xi = Xr + XR * kWavePanel;
  double* pb = Xr + (CPLX ? 2 : 1) * XR * kWavePanel;
  unsigned char* s_op = (unsigned char*)(pb + XR);
  short* s_path = (short*)(s_op + kMaxOps);
  // workgroup tables
  int* s_dim = (int*)((char*)lds + 4 * per_wave);
  int* s_eoff = s_dim + NS;
  short* s_next = (short*)(s_eoff + NS);
  const bool next_in_lds = I.next_lds != 0;
  for (int i = tid; i < NS; i += 256) {
    s_dim[i] = I.dim[i];
    s_eoff[i] = I.eoff[i];
  }
  if (next_in_lds)
    for (int i = tid; i < NS * I.nops; i += 256) s_next[i] = (short)I.next[i];
  __syncthreads();

  const long long total = B.cfg_off[B.n_cfg];
  for (;;) {
    long long w = 0;
    if (lane == 0) w = (long long)atomicAdd(B.counter, 1u);
    w = __shfl(w, 0);
    if (w >= total) break;

    int lo = 0, hi = B.n_cfg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.cfg_off[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const int local = (int)(w - B.cfg_off[c]);
    const StrRec* recs = B.rec + (long long)c * NS;
    lo = 0;
    hi = NS - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
    }
    const StrRec R = recs[lo];
    const int col0 = (local - R.loc_off) * kWavePanel;
    const int ncols = min(kWavePanel, R.width - col0);
    const int G = __builtin_amdgcn_readfirstlane((ncols + 3) >> 2);  // column groups of four, uniform
    const long long base = B.offsets[c];
    const int n = (int)(B.offsets[c + 1] - base);
    const double* tau = B.tau + base;
    const int* opg = B.op + base;

    PanelRes out;
    out.re = out.im = out.e2 = 0.0;
    const int s0 = R.q_start;
    constexpr bool lazy = LAZY;
    unsigned long long ucur = lazy ? lazy_initial(R, local) : 0;
    bool dead = false;
    if (n == 0) {
      // partition-function string: trace of the diagonal propagator
      const double* e = I.esh + s_eoff[s0];
      double v = (lane < ncols) ? exp(-I.beta * e[col0 + lane]) : 0.0;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      out.re = v;
    } else {
      // string in LDS: rotated operator codes, then the visited sectors
      for (int t = lane; t < n; t += 64) s_op[t] = (unsigned char)opg[(R.jstar + t) % n];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) {
        int q = s0;
        s_path[0] = (short)q;
        for (int t = 0; t < n; ++t) {
          q = next_in_lds ? s_next[q * I.nops + s_op[t]] : I.next[q * I.nops + s_op[t]];
          s_path[t + 1] = (short)q;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();

      int ce[2] = {0, 0};  // power of two of columns g*4 + l3
      long long boff_next = I.boff[s0 * I.nops + s_op[0]];
      int rj_prev = 0;  // lazy: the configuration's rejection flag, read one step earlier
      for (int t = 0; t < n - 1; ++t) {
        if (lazy) {
          // the flag read at the previous step decides; this step's read is
          // issued now and waited for only at the next step, behind this
          // step's products
          if (__shfl(rj_prev, 0)) {
            dead = true;
            break;
          }
          rj_prev = (lane == 0) ? (int)lazy_rejected(B, c) : 0;
        }
        const int s = s_path[t], s2 = s_path[t + 1];
        const int d_in = s_dim[s], d_out = s_dim[s2];
        const int ld = (d_out + 15) & ~15;
        const int ntiles = ld >> 4;
        const double* Fr = I.pool + boff_next;
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        boff_next = I.boff[s2 * I.nops + s_op[t + 1]];
        // nonzero-tile masks of this step's block, loaded before the propagator
        // work below so that their latency is hidden behind it
        const uint4* tmv = (const uint4*)(I.tmask + (long long)__builtin_amdgcn_readfirstlane(s * I.nops + s_op[t]) *
                                                         kWaveTiles);
        const uint4 mlo = tmv[0], mhi = tmv[1];
        const int p1 = (R.jstar + t + 1) % n;  // position in front of the next operator
        const double dt2 = p1 ? tau[p1] - tau[p1 - 1] : tau[0] + I.beta - tau[n - 1];
        {
          const double* e = I.esh + s_eoff[s2];
          for (int r = lane; r < ld; r += 64) pb[r] = (r < d_out) ? exp(-dt2 * e[r]) : 0.0;
        }
        double acc_r[kWaveTiles][2], acc_i[kWaveTiles][2];
#pragma unroll
        for (int tt = 0; tt < kWaveTiles; ++tt) acc_r[tt][0] = acc_r[tt][1] = acc_i[tt][0] = acc_i[tt][1] = 0.0;
        if (t == 0) {
          const int p0 = R.jstar;
          const double dt0 = p0 ? tau[p0] - tau[p0 - 1] : tau[0] + I.beta - tau[n - 1];
          const double* e0 = I.esh + s_eoff[s];
#pragma unroll
          for (int g = 0; g < 2; ++g) {
            const int cc = g * 4 + l3;
            if (cc < ncols) {
              const int k = col0 + cc;
              const double p = exp(-dt0 * e0[k]);
#pragma unroll
              for (int tt = 0; tt < kWaveTiles; ++tt) {
                if (tt < ntiles) {
                  const long long a = (long long)k * ld + tt * 16 + orow;
                  acc_r[tt][g] = Fr[a] * p;
                  if (CPLX) acc_i[tt][g] = Fi[a] * p;
                }
              }
            }
          }
        } else {
          // only the 16 x 4 tiles of the block that hold a nonzero are multiplied
          // (the others add exact zeros): row tile by row tile, its nonzero
          // k-steps in ascending order (the accumulation order of the dense
          // loop), kTileBatch at a time so that their loads are in flight together.
          // The block's masks are wavefront-uniform.
          const unsigned int mw[kWaveTiles] = {mlo.x, mlo.y, mlo.z, mlo.w, mhi.x, mhi.y, mhi.z, mhi.w};
#pragma unroll
          for (int tt = 0; tt < kWaveTiles; ++tt) {
            if (tt >= ntiles) continue;
            unsigned int m = __builtin_amdgcn_readfirstlane(mw[tt]);
            while (m) {
              // the batch's k-steps; unused slots repeat the first one, so that
              // every load of the batch is issued together (and stays in bounds)
              int kq[kTileBatch];
              kq[0] = __builtin_ctz(m);
              m &= m - 1;
              int nb = 1;
#pragma unroll
              for (int j2 = 1; j2 < kTileBatch; ++j2) {
                kq[j2] = kq[0];
                if (m) {
                  kq[j2] = __builtin_ctz(m);
                  m &= m - 1;
                  ++nb;
                }
              }
              double ar[kTileBatch], ai[kTileBatch], b0r[kTileBatch], b1r[kTileBatch], b0i[kTileBatch], b1i[kTileBatch];
#pragma unroll
              for (int j2 = 0; j2 < kTileBatch; ++j2) {
                const int krow = kq[j2] * 4 + lq;
                const long long a = (long long)krow * ld + tt * 16 + ln;
                ar[j2] = Fr[a];
                ai[j2] = CPLX ? Fi[a] : 0.0;
                b0r[j2] = Xr[krow * kWavePanel + l3];
                b1r[j2] = Xr[krow * kWavePanel + 4 + l3];
                b0i[j2] = CPLX ? Xi[krow * kWavePanel + l3] : 0.0;
                b1i[j2] = CPLX ? Xi[krow * kWavePanel + 4 + l3] : 0.0;
              }
#pragma unroll
              for (int j2 = 0; j2 < kTileBatch; ++j2) {
                if (j2 < nb) {
                  acc_r[tt][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[j2], b0r[j2], acc_r[tt][0], 0, 0, 0);
                  if (CPLX) {
                    acc_r[tt][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(-ai[j2], b0i[j2], acc_r[tt][0], 0, 0, 0);
                    acc_i[tt][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[j2], b0i[j2], acc_i[tt][0], 0, 0, 0);
                    acc_i[tt][0] = __builtin_amdgcn_mfma_f64_4x4x4f64(ai[j2], b0r[j2], acc_i[tt][0], 0, 0, 0);
                  }
                  if (G > 1) {
                    acc_r[tt][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[j2], b1r[j2], acc_r[tt][1], 0, 0, 0);
                    if (CPLX) {
                      acc_r[tt][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(-ai[j2], b1i[j2], acc_r[tt][1], 0, 0, 0);
                      acc_i[tt][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(ar[j2], b1i[j2], acc_i[tt][1], 0, 0, 0);
                      acc_i[tt][1] = __builtin_amdgcn_mfma_f64_4x4x4f64(ai[j2], b1r[j2], acc_i[tt][1], 0, 0, 0);
                    }
                  }
                }
              }
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // propagator in front of the next operator, per-column max, rescale
        double cm0 = 0.0, cm1 = 0.0;
#pragma unroll
        for (int tt = 0; tt < kWaveTiles; ++tt) {
          if (tt < ntiles) {
            const double p = pb[tt * 16 + orow];
            acc_r[tt][0] *= p;
            acc_r[tt][1] *= p;
            cm0 = fmax(cm0, fabs(acc_r[tt][0]));
            cm1 = fmax(cm1, fabs(acc_r[tt][1]));
            if (CPLX) {
              acc_i[tt][0] *= p;
              acc_i[tt][1] *= p;
              cm0 = fmax(cm0, fabs(acc_i[tt][0]));
              cm1 = fmax(cm1, fabs(acc_i[tt][1]));
            }
          }
        }
        for (int off = 4; off < 64; off <<= 1) {
          cm0 = fmax(cm0, __shfl_xor(cm0, off));
          cm1 = fmax(cm1, __shfl_xor(cm1, off));
        }
        int e0 = 0, e1 = 0;
        if (cm0 > 0.0) frexp(cm0, &e0);
        if (cm1 > 0.0) frexp(cm1, &e1);
        ce[0] += e0;
        ce[1] += e1;
        const double sc0 = ldexp(1.0, -e0), sc1 = ldexp(1.0, -e1);
#pragma unroll
        for (int tt = 0; tt < kWaveTiles; ++tt) {
          if (tt < ntiles) {
            const int m = tt * 16 + orow;
            Xr[m * kWavePanel + l3] = acc_r[tt][0] * sc0;
            Xr[m * kWavePanel + 4 + l3] = acc_r[tt][1] * sc1;
            if (CPLX) {
              Xi[m * kWavePanel + l3] = acc_i[tt][0] * sc0;
              Xi[m * kWavePanel + 4 + l3] = acc_i[tt][1] * sc1;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lazy && (t & 3) == 3) {
          // Frobenius norm of the panel: columns l3 and 4 + l3 of every lane
          double q0 = 0.0, q1 = 0.0;
#pragma unroll
          for (int tt = 0; tt < kWaveTiles; ++tt) {
            if (tt < ntiles) {
              const double a0 = acc_r[tt][0] * sc0, a1 = acc_r[tt][1] * sc1;
              q0 += a0 * a0;
              q1 += a1 * a1;
              if (CPLX) {
                const double b0 = acc_i[tt][0] * sc0, b1 = acc_i[tt][1] * sc1;
                q0 += b0 * b0;
                q1 += b1 * b1;
              }
            }
          }
          for (int off = 4; off < 64; off <<= 1) {
            q0 += __shfl_xor(q0, off);
            q1 += __shfl_xor(q1, off);
          }
          const double A0 = q0 > 0.0 ? log(q0) + 2.0 * ce[0] * 0.69314718055994530942 : -INFINITY;
          const double A1 = q1 > 0.0 ? log(q1) + 2.0 * ce[1] * 0.69314718055994530942 : -INFINITY;
          const double mA = fmax(A0, A1);
          const double lane_sum = (mA == -INFINITY) ? -INFINITY : mA + log(exp(A0 - mA) + exp(A1 - mA));
          const double logF2 = logsumexp_quad(lane_sum);
          int rj = 0;
          if (lane == 0 && logF2 > -INFINITY)
            rj = lazy_update(B, c, &ucur, 0.5 * (logF2 + log((double)ncols)) - R.L);
          ucur = __shfl(ucur, 0);
          if (__shfl(rj, 0)) {
            dead = true;
            break;
          }
        }
      }

      // last operator: diagonal of F * X; lane = column (l & 7) x k-partial (l >> 3)
      if (!dead) {
        const int s = s_path[n - 1];
        const int d_in = s_dim[s];
        const int ld = (s_dim[s_path[n]] + 15) & ~15;
        const double* Fr = I.pool + boff_next;
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        const int cc = lane & 7;
        double sr = 0.0, si = 0.0;
        if (cc < ncols) {
          for (int k = lane >> 3; k < d_in; k += 8) {
            const long long a = (long long)k * ld + col0 + cc;
            const double fr = Fr[a], xr = Xr[k * kWavePanel + cc];
            if (CPLX) {
              const double fi = Fi[a], xi = Xi[k * kWavePanel + cc];
              sr += fr * xr - fi * xi;
              si += fr * xi + fi * xr;
            } else {
              sr += fr * xr;
            }
          }
        }
        for (int off = 8; off < 64; off <<= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        // exponent of column cc lives in lanes with l3 == cc % 4 (entry cc / 4)
        const int ea = __shfl(ce[0], cc & 3), eb = __shfl(ce[1], cc & 3);
        const int ec = (cc < 4) ? ea : eb;
        const bool live = cc < ncols && (sr != 0.0 || si != 0.0);
        int emax = live ? ec : INT_MIN;
        for (int off = 1; off < 8; off <<= 1) emax = max(emax, __shfl_xor(emax, off));
        if (emax != INT_MIN) {
          const double f = live ? ldexp(1.0, ec - emax) : 0.0;
          double vr = sr * f, vi = si * f;
          for (int off = 1; off < 8; off <<= 1) {
            vr += __shfl_xor(vr, off);
            vi += __shfl_xor(vi, off);
          }
          out.re = vr;
          out.im = vi;
          out.e2 = (double)emax;
        }
        if (lazy && lane == 0) {
          const double a = hypot(out.re, out.im);
          lazy_update(B, c, &ucur, a > 0.0 ? log(a) + out.e2 * 0.69314718055994530942 - R.L : -INFINITY);
        }
      }
    }
    if (lane == 0) B.res[w] = out;
  }
}

// ---------------------------------------------------------------------------
// chain, streaming (sectors too large for an LDS-resident panel)
// ---------------------------------------------------------------------------
// One workgroup of 16 wavefronts per panel of 16 columns; the carried matrix
// lives in a per-workgroup pair of global buffers (L2 resident).  Each
// wavefront computes groups of kBigGroup 16-row tiles at a time over the
// whole K range (operand B loaded once per group), applies the next
// propagator and keeps a running per-column max; the column rescale of a
// step is applied when the next step loads its operand (exact power of two,
// exponents accumulated per column).
constexpr int kBigWaves = 16;
constexpr int kBigGroup = 4;

__host__ __device__ constexpr size_t big_lds_bytes(int xr, int n_sec) {
  return 8 * ((size_t)xr + 2 * kBigWaves * kPanel + kMaxOps + kPanel * 2) + 4 * (2 * (size_t)n_sec) +
         2 * (2 * (size_t)kMaxOps + 2) + 64;
}

template <bool CPLX, bool LAZY>
__global__ __launch_bounds__(kBigWaves * 64) void k_chain_big(DevImp I, BatchArgs B, double* xbuf) {
  extern __shared__ double lds[];
  constexpr int NT = kBigWaves * 64;
  constexpr int GRP = CPLX ? 2 : kBigGroup;  // row tiles per pass (register budget)
  const int XR = I.xrows;
  const int NS = I.n_sec;
  double* pb = lds;                          // [XR] propagator in front of the next operator
  double* cmax = pb + XR;                    // [kBigWaves][16]
  double* s_dt = cmax + kBigWaves * kPanel;  // [kMaxOps]
  double* s_red = s_dt + kMaxOps;            // [2][16] close sums
  double* cmaxi = s_red + 2 * kPanel;        // [kBigWaves][16] close partials, imaginary part
  int* s_dim = (int*)(cmaxi + kBigWaves * kPanel);
  int* s_eoff = s_dim + NS;
  short* s_op = (short*)(s_eoff + NS);       // [kMaxOps]
  short* s_path = s_op + kMaxOps;            // [kMaxOps + 1]
  __shared__ long long s_w;
  __shared__ int s_cexp[kPanel];             // accumulated power of two per column
  __shared__ int s_pend[kPanel];             // rescale pending from the previous step
  __shared__ double s_csq[kBigWaves][kPanel];  // lazy: per-wavefront column sums of squares
  __shared__ int s_rej;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  // this workgroup's buffers: two copies of X (re plane, then im plane)
  const size_t plane = (size_t)XR * kPanel;
  double* X0 = xbuf + (size_t)blockIdx.x * 2 * (CPLX ? 2 : 1) * plane;
  double* X1 = X0 + (CPLX ? 2 : 1) * plane;

  for (int i = tid; i < NS; i += NT) {
    s_dim[i] = I.dim[i];
    s_eoff[i] = I.eoff[i];
  }
  const long long total = B.cfg_off[B.n_cfg];
  for (;;) {
    if (tid == 0) s_w = (long long)atomicAdd(B.counter, 1u);
    __syncthreads();
    const long long w = s_w;
    if (w >= total) break;
    int lo = 0, hi = B.n_cfg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (B.cfg_off[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const int c = lo;
    const int local = (int)(w - B.cfg_off[c]);
    const StrRec* recs = B.rec + (long long)c * NS;
    lo = 0;
    hi = NS - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
    }
    const StrRec R = recs[lo];
    const int col0 = (local - R.loc_off) * kPanel;
    const int ncols = min(kPanel, R.width - col0);
    const long long base = B.offsets[c];
    const int n = (int)(B.offsets[c + 1] - base);
    for (int t = tid; t < n; t += NT) {
      const int p = (R.jstar + t) % n;
      s_op[t] = (short)B.op[base + p];
      s_dt[t] = p ? B.tau[base + p] - B.tau[base + p - 1] : B.tau[base] + I.beta - B.tau[base + n - 1];
    }
    if (tid < kPanel) {
      s_cexp[tid] = 0;
      s_pend[tid] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      int q = R.q_start;
      s_path[0] = (short)q;
      for (int t = 0; t < n; ++t) {
        q = I.next[q * I.nops + s_op[t]];
        s_path[t + 1] = (short)q;
      }
    }
    __syncthreads();

    PanelRes out;
    out.re = out.im = out.e2 = 0.0;
    constexpr bool lazy = LAZY;
    unsigned long long ucur = lazy ? lazy_initial(R, local) : 0;  // used by thread 0
    bool dead = false;
    if (n == 0) {
      if (tid == 0) {
        const double* e = I.esh + s_eoff[R.q_start];
        double sum = 0.0;
        for (int cc = 0; cc < ncols; ++cc) sum += exp(-I.beta * e[col0 + cc]);
        out.re = sum;
      }
    } else {
      double* Xin = X1;
      double* Xout = X0;
      for (int t = 0; t < n - 1; ++t) {
        if (lazy) {
          if (tid == 0) s_rej = lazy_rejected(B, c) ? 1 : 0;
          __syncthreads();
          if (s_rej) {
            dead = true;
            break;
          }
        }
        const int s = s_path[t], s2 = s_path[t + 1];
        const int d_in = s_dim[s], d_out = s_dim[s2];
        const int ld = (d_out + 15) & ~15;
        const int ntiles = ld >> 4;
        const long long bo = I.boff[s * I.nops + s_op[t]];
        const double* Fr = I.pool + bo;
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        {
          const double dt2 = s_dt[t + 1];
          const double* e = I.esh + s_eoff[s2];
          for (int r = tid; r < ld; r += NT) pb[r] = (r < d_out) ? exp(-dt2 * e[r]) : 0.0;
        }
        // scale of the input columns (rescale deferred from the previous step)
        const double bsc = ldexp(1.0, -s_pend[ln]);
        const double* e0 = I.esh + s_eoff[s];
        const double p0 = (t == 0 && ln < ncols) ? exp(-s_dt[0] * e0[col0 + ln]) : 0.0;
        __syncthreads();
        double cm = 0.0, csq = 0.0;
        for (int g0 = wave * GRP; g0 < ntiles; g0 += kBigWaves * GRP) {
          dbl4 acc_r[GRP], acc_i[GRP];
#pragma unroll
          for (int g = 0; g < GRP; ++g) {
            acc_r[g] = dbl4{0.0, 0.0, 0.0, 0.0};
            acc_i[g] = dbl4{0.0, 0.0, 0.0, 0.0};
          }
          if (t == 0) {
            if (ln < ncols) {
              const int k = col0 + ln;
#pragma unroll
              for (int g = 0; g < GRP; ++g) {
                if (g0 + g < ntiles) {
#pragma unroll
                  for (int i = 0; i < 4; ++i) {
                    const long long a = (long long)k * ld + (g0 + g) * 16 + 4 * i + lq;
                    acc_r[g][i] = Fr[a] * p0;
                    if (CPLX) acc_i[g][i] = Fi[a] * p0;
                  }
                }
              }
            }
          } else {
            const int ksteps = (d_in + 3) >> 2;
            for (int kc = 0; kc < ksteps; ++kc) {
              const int krow = kc * 4 + lq;
              const double br = Xin[krow * kPanel + ln] * bsc;
              const double bi = CPLX ? Xin[plane + krow * kPanel + ln] * bsc : 0.0;
#pragma unroll
              for (int g = 0; g < GRP; ++g) {
                if (g0 + g < ntiles) {
                  const long long a = (long long)krow * ld + (g0 + g) * 16 + ln;
                  const double ar = Fr[a];
                  acc_r[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, acc_r[g], 0, 0, 0);
                  if (CPLX) {
                    const double ai = Fi[a];
                    acc_r[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, bi, acc_r[g], 0, 0, 0);
                    acc_i[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, acc_i[g], 0, 0, 0);
                    acc_i[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, br, acc_i[g], 0, 0, 0);
                  }
                }
              }
            }
          }
#pragma unroll
          for (int g = 0; g < GRP; ++g) {
            if (g0 + g < ntiles) {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int m = (g0 + g) * 16 + 4 * i + lq;
                const double p = pb[m];
                const double vr = acc_r[g][i] * p;
                Xout[m * kPanel + ln] = vr;
                cm = fmax(cm, fabs(vr));
                if (lazy) csq += vr * vr;
                if (CPLX) {
                  const double vi = acc_i[g][i] * p;
                  Xout[plane + m * kPanel + ln] = vi;
                  cm = fmax(cm, fabs(vi));
                  if (lazy) csq += vi * vi;
                }
              }
            }
          }
        }
        cm = fmax(cm, __shfl_xor(cm, 16));
        cm = fmax(cm, __shfl_xor(cm, 32));
        csq += __shfl_xor(csq, 16);
        csq += __shfl_xor(csq, 32);
        if (lane < 16) {
          cmax[wave * kPanel + lane] = cm;
          s_csq[wave][lane] = csq;
        }
        __threadfence_block();
        __syncthreads();
        if (tid < kPanel) {
          double M = 0.0, Q = 0.0;
          for (int w2 = 0; w2 < kBigWaves; ++w2) {
            M = fmax(M, cmax[w2 * kPanel + tid]);
            Q += s_csq[w2][tid];
          }
          // lazy: log of this column's squared norm (X unscaled, exponents before this step)
          if (lazy) s_red[tid] = Q > 0.0 ? log(Q) + 2.0 * s_cexp[tid] * 0.69314718055994530942 : -INFINITY;
          int e = 0;
          if (M > 0.0) frexp(M, &e);
          s_pend[tid] = e;        // applied by the next load of X
          s_cexp[tid] += e;
        }
        __syncthreads();
        if (lazy && (t & 3) == 3) {
          if (tid == 0) {
            double mx = -INFINITY;
            for (int j = 0; j < kPanel; ++j) mx = fmax(mx, s_red[j]);
            int rj = 0;
            if (mx > -INFINITY) {
              double sum = 0.0;
              for (int j = 0; j < kPanel; ++j) sum += exp(s_red[j] - mx);
              const double logF2 = mx + log(sum);
              rj = lazy_update(B, c, &ucur, 0.5 * (logF2 + log((double)ncols)) - R.L) ? 1 : 0;
            }
            s_rej = rj;
          }
          __syncthreads();
          if (s_rej) {
            dead = true;
            break;
          }
        }
        double* tmp = Xin;
        Xin = Xout;
        Xout = tmp;
      }
      // last operator: diagonal of F * (X * 2^-pend), rows col0 .. col0+ncols
      if (!dead) {
        const int s = s_path[n - 1];
        const int d_in = s_dim[s];
        const int ld = (s_dim[s_path[n]] + 15) & ~15;
        const double* Fr = I.pool + I.boff[s * I.nops + s_op[n - 1]];
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        const int cc = tid & 15;
        const double bsc = ldexp(1.0, -s_pend[cc]);
        double sr = 0.0, si = 0.0;
        if (cc < ncols) {
          for (int k = tid >> 4; k < d_in; k += NT / 16) {
            const long long a = (long long)k * ld + col0 + cc;
            const double fr = Fr[a], xr = Xin[k * kPanel + cc] * bsc;
            if (CPLX) {
              const double fi = Fi[a], xi = Xin[plane + k * kPanel + cc] * bsc;
              sr += fr * xr - fi * xi;
              si += fr * xi + fi * xr;
            } else {
              sr += fr * xr;
            }
          }
        }
        // reduce over the 64 k-partials of every column: wavefront, then LDS
        for (int off = 16; off < 64; off <<= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        if (lane < 16) {
          cmax[wave * kPanel + lane] = sr;
          cmaxi[wave * kPanel + lane] = si;
        }
        __syncthreads();
        if (tid == 0) {
          int emax = INT_MIN;
          for (int j = 0; j < ncols; ++j) {
            double vr = 0.0, vi = 0.0;
            for (int w2 = 0; w2 < kBigWaves; ++w2) {
              vr += cmax[w2 * kPanel + j];
              vi += cmaxi[w2 * kPanel + j];
            }
            s_red[j] = vr;
            s_red[kPanel + j] = vi;
            if (vr != 0.0 || vi != 0.0) emax = max(emax, s_cexp[j]);
          }
          if (emax != INT_MIN) {
            double vr = 0.0, vi = 0.0;
            for (int j = 0; j < ncols; ++j) {
              const double f = ldexp(1.0, s_cexp[j] - emax);
              vr += s_red[j] * f;
              vi += s_red[kPanel + j] * f;
            }
            out.re = vr;
            out.im = vi;
            out.e2 = (double)emax;
          }
          if (lazy) {
            const double a = hypot(out.re, out.im);
            lazy_update(B, c, &ucur, a > 0.0 ? log(a) + out.e2 * 0.69314718055994530942 - R.L : -INFINITY);
          }
        }
      }
    }
    if (tid == 0) B.res[w] = out;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// combine
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_combine(DevImp I, BatchArgs B) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= B.n_cfg) return;
  ctr_value v;
  v.re = v.im = v.log_scale = 0.0;
  v.log_abs = -INFINITY;
  int flags = B.cfg_flags[c];
  if (B.log_thr != nullptr && B.cfg_rej[c]) flags |= CTR_FLAG_REJECTED;
  v.flags = flags;
  v.n_strings = B.cfg_nstr[c];
  v.log_bound = B.cfg_logB[c];
  if (!(flags & (CTR_FLAG_INVALID | CTR_FLAG_REJECTED | CTR_FLAG_ZERO))) {
    const double ln2 = 0.69314718055994530942;
    const StrRec* recs = B.rec + (long long)c * I.n_sec;
    const PanelRes* res = B.res + B.cfg_off[c];
    double lmax = -INFINITY;
    for (int q = 0; q < I.n_sec; ++q) {
      const StrRec R = recs[q];
      for (int p = 0; p < R.n_panels; ++p) {
        const PanelRes P = res[R.loc_off + p];
        if (P.re != 0.0 || P.im != 0.0) lmax = fmax(lmax, P.e2 * ln2 - R.L);
      }
    }
    if (lmax > -INFINITY) {
      double sr = 0.0, si = 0.0, sa = 0.0;
      for (int q = 0; q < I.n_sec; ++q) {
        const StrRec R = recs[q];
        for (int p = 0; p < R.n_panels; ++p) {
          const PanelRes P = res[R.loc_off + p];
          if (P.re != 0.0 || P.im != 0.0) {
            const double f = exp(P.e2 * ln2 - R.L - lmax);
            sr += P.re * f;
            si += P.im * f;
            sa += hypot(P.re, P.im) * f;
          }
        }
      }
      v.re = sr;
      v.im = si;
      v.log_scale = lmax - I.beta * I.E0;
      v.log_abs = log(sa) + v.log_scale;
    }
  }
  B.out[c] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_plan(const DevImp& imp, const BatchArgs& b, hipStream_t stream) {
  if (b.n_cfg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan, dim3(b.n_cfg), dim3(kPlanThreads), 0, stream, imp, b);
  return hipGetLastError();
}

hipError_t launch_scan(const BatchArgs& b, hipStream_t stream) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, stream, b);
  return hipGetLastError();
}

hipError_t launch_combine(const DevImp& imp, const BatchArgs& b, hipStream_t stream) {
  if (b.n_cfg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3((b.n_cfg + 255) / 256), dim3(256), 0, stream, imp, b);
  return hipGetLastError();
}

namespace {

struct Variant {
  const void* fn;
  int nw;
  int maxt;
  bool cplx;
};

template <bool CPLX, int NW, int MAXT>
Variant make_variant(int slices) {
  return Variant{slices == 7   ? reinterpret_cast<const void*>(&k_chain<CPLX, NW, MAXT, 7>)
                 : slices == 6 ? reinterpret_cast<const void*>(&k_chain<CPLX, NW, MAXT, 6>)
                               : reinterpret_cast<const void*>(&k_chain<CPLX, NW, MAXT, 0>),
                 NW, MAXT, CPLX};
}

bool pick_variant(const DevImp& imp, int split, Variant* v) {
  const int tiles = imp.xrows / 16;
  if (imp.is_complex) {
    if (tiles <= 8) *v = make_variant<true, 4, 2>(split);
    else if (tiles <= 16) *v = make_variant<true, 8, 2>(split);
    else if (tiles <= 32) *v = make_variant<true, 8, 4>(split);
    else if (tiles <= 64) *v = make_variant<true, 16, 4>(split);
    else return false;
  } else {
    if (tiles <= 8) *v = make_variant<false, 4, 2>(split);
    else if (tiles <= 16) *v = make_variant<false, 8, 2>(split);
    else if (tiles <= 32) *v = make_variant<false, 8, 4>(split);
    else if (tiles <= 64) *v = make_variant<false, 16, 4>(split);
    else return false;
  }
  return true;
}

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

size_t chain_lds_bytes(const DevImp& imp) {
  Variant v;
  if (!pick_variant(imp, false, &v)) return 0;
  const int ne = imp.next_lds ? imp.n_sec * imp.nops : 0;
  const int xr = imp.xrows, ns = imp.n_sec;
  return v.cplx ? (v.nw == 4 ? chain_lds_bytes_t<true, 4>(xr, ns, ne)
                  : v.nw == 8 ? chain_lds_bytes_t<true, 8>(xr, ns, ne)
                              : chain_lds_bytes_t<true, 16>(xr, ns, ne))
                : (v.nw == 4 ? chain_lds_bytes_t<false, 4>(xr, ns, ne)
                  : v.nw == 8 ? chain_lds_bytes_t<false, 8>(xr, ns, ne)
                              : chain_lds_bytes_t<false, 16>(xr, ns, ne));
}

int chain_max_rows(int is_complex) { return is_complex ? 576 : 1024; }

int chain_grid(const DevImp& imp, int device, int split, size_t* lds_bytes) {
  Variant v;
  if (!pick_variant(imp, split, &v)) return 0;
  const size_t bytes = chain_lds_bytes(imp);
  if (lds_bytes) *lds_bytes = bytes;
  if (bytes > kMaxLds) return 0;
  if (hipFuncSetAttribute(v.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, v.nw * 64, bytes) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (per_cu <= 0) return 0;
  return per_cu * cus;
}

int wave_grid(const DevImp& imp, int device, size_t* lds_bytes, bool lazy) {
  if (imp.xrows > kWaveTiles * 16) return 0;
  const int ne = imp.next_lds ? imp.n_sec * imp.nops : 0;
  const size_t bytes = imp.is_complex ? wave_lds_bytes<true>(imp.xrows, imp.n_sec, ne)
                                      : wave_lds_bytes<false>(imp.xrows, imp.n_sec, ne);
  if (lds_bytes) *lds_bytes = bytes;
  if (bytes > kMaxLds) return 0;
  const void* fns[2] = {imp.is_complex ? reinterpret_cast<const void*>(&k_chain_wave<true, false>)
                                        : reinterpret_cast<const void*>(&k_chain_wave<false, false>),
                        imp.is_complex ? reinterpret_cast<const void*>(&k_chain_wave<true, true>)
                                        : reinterpret_cast<const void*>(&k_chain_wave<false, true>)};
  // the plain and the lazy form are sized apart (the plain one runs four
  // workgroups per CU, the lazy one, with its bound bookkeeping, three);
  // neither is offered unless both can run
  int per_cu[2] = {0, 0};
  for (int v = 0; v < 2; ++v) {
    if (hipFuncSetAttribute(fns[v], hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[v], fns[v], 256, bytes) != hipSuccess) return 0;
  }
  if (per_cu[0] <= 0 || per_cu[1] <= 0) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu[lazy ? 1 : 0] * cus;
}

hipError_t launch_chain_wave(const DevImp& imp, const BatchArgs& b, int grid, hipStream_t stream) {
  size_t bytes = 0;
  const int ne = imp.next_lds ? imp.n_sec * imp.nops : 0;
  bytes = imp.is_complex ? wave_lds_bytes<true>(imp.xrows, imp.n_sec, ne)
                         : wave_lds_bytes<false>(imp.xrows, imp.n_sec, ne);
  const bool lazy = b.log_thr != nullptr;
  const void* fn = imp.is_complex ? (lazy ? reinterpret_cast<const void*>(&k_chain_wave<true, true>)
                                          : reinterpret_cast<const void*>(&k_chain_wave<true, false>))
                                  : (lazy ? reinterpret_cast<const void*>(&k_chain_wave<false, true>)
                                          : reinterpret_cast<const void*>(&k_chain_wave<false, false>));
  void* args[] = {const_cast<DevImp*>(&imp), const_cast<BatchArgs*>(&b)};
  return hipLaunchKernel(fn, dim3(grid), dim3(256), args, bytes, stream);
}

int big_grid(const DevImp& imp, int device, size_t* lds_bytes) {
  const size_t bytes = big_lds_bytes(imp.xrows, imp.n_sec);
  if (lds_bytes) *lds_bytes = bytes;
  if (bytes > kMaxLds) return 0;
  const void* fns[2] = {imp.is_complex ? reinterpret_cast<const void*>(&k_chain_big<true, false>)
                                        : reinterpret_cast<const void*>(&k_chain_big<false, false>),
                        imp.is_complex ? reinterpret_cast<const void*>(&k_chain_big<true, true>)
                                        : reinterpret_cast<const void*>(&k_chain_big<false, true>)};
  int per_cu = 1 << 30;
  for (const void* fn : fns) {
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) return 0;
    int k = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, fn, kBigWaves * 64, bytes) != hipSuccess) return 0;
    per_cu = std::min(per_cu, k);
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return per_cu > 0 ? per_cu * cus : 0;
}

size_t big_xbuf_doubles(const DevImp& imp, int grid) {
  return (size_t)grid * 2 * (imp.is_complex ? 2 : 1) * (size_t)imp.xrows * kPanel;
}

hipError_t launch_chain_big(const DevImp& imp, const BatchArgs& b, double* xbuf, int grid, hipStream_t stream) {
  const size_t bytes = big_lds_bytes(imp.xrows, imp.n_sec);
  const bool lazy = b.log_thr != nullptr;
  const void* fn = imp.is_complex ? (lazy ? reinterpret_cast<const void*>(&k_chain_big<true, true>)
                                          : reinterpret_cast<const void*>(&k_chain_big<true, false>))
                                  : (lazy ? reinterpret_cast<const void*>(&k_chain_big<false, true>)
                                          : reinterpret_cast<const void*>(&k_chain_big<false, false>));
  void* args[] = {const_cast<DevImp*>(&imp), const_cast<BatchArgs*>(&b), &xbuf};
  return hipLaunchKernel(fn, dim3(grid), dim3(kBigWaves * 64), args, bytes, stream);
}

hipError_t launch_chain(const DevImp& imp, const BatchArgs& b, int split, int grid, hipStream_t stream) {
  Variant v;
  if (!pick_variant(imp, split, &v) || grid <= 0) return hipErrorInvalidValue;
  const size_t bytes = chain_lds_bytes(imp);
  void* args[] = {const_cast<DevImp*>(&imp), const_cast<BatchArgs*>(&b)};
  return hipLaunchKernel(v.fn, dim3(grid), dim3(v.nw * 64), args, bytes, stream);
}

}  // namespace ctr
