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
//              MFMA 16x16x4 block products, and a per-column power-of-two
//              rescale from wavefront max-reductions; the last operator only
//              contributes the diagonal of F * X.
//   k_combine  one thread per configuration: merges the (mantissa, exponent)
//              panel results of all strings in a fixed order.
#include <math.h>

#include "ctrace_internal.h"

namespace ctr {

typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double dtp(const double* tau, int n, int p, double beta) {
  // imaginary-time gap in front of operator p; position 0 also carries the
  // gap after the last operator (the two end propagators merge by cyclicity)
  return p ? tau[p] - tau[p - 1] : tau[0] + beta - tau[n - 1];
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
        R.n_panels = (best + kPanel - 1) / kPanel;
        R.L = L;
        R.logB = log((double)best) - L + logn;
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
  __syncthreads();
  for (int off = kPlanThreads / 2; off > 0; off >>= 1) {
    if (t < off) {
      s_red[t] += s_red[t + off];
      s_scan[t] += s_scan[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    const int nstr = s_scan[0];
    const double logB = nstr > 0 ? gmax + log(s_red[0]) - I.beta * I.E0 : -INFINITY;
    int flags = bad ? CTR_FLAG_INVALID : 0;
    int cnt = bad ? 0 : total;
    if (!bad && nstr == 0) flags |= CTR_FLAG_ZERO;
    if (!bad && nstr > 0 && B.log_thr != nullptr && logB < B.log_thr[c]) {
      flags |= CTR_FLAG_REJECTED;
      cnt = 0;
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
__host__ __device__ constexpr size_t chain_lds_doubles(int xr) {
  return (size_t)(CPLX ? 2 : 1) * xr * kPanel + 2 * (size_t)xr + NW * kPanel + (CPLX ? 2 : 1) * NW * 64 + kPanel;
}

template <bool CPLX, int NW, int MAXT>
__global__ __launch_bounds__(NW * 64) void k_chain(DevImp I, BatchArgs B) {
  extern __shared__ double lds[];
  constexpr int NT = NW * 64;
  const int XR = I.xrows;
  double* Xr = lds;                                    // [XR][16]
  double* Xi = lds + XR * kPanel;                      // [XR][16], complex only
  double* pa = lds + (CPLX ? 2 : 1) * XR * kPanel;     // propagator at the start position
  double* pb = pa + XR;                                // propagator in front of the next operator
  double* cmax = pb + XR;                              // [NW][16]
  double* red = cmax + NW * kPanel;                    // [NT] (x2 complex)
  int* colexp = (int*)(red + (CPLX ? 2 : 1) * NT);     // [16] per-column power of two
  __shared__ long long s_w;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ln = lane & 15;  // column of the 16x16 tile held by this lane
  const int lq = lane >> 4;  // row group: D item i of this lane is row 4*i + lq
  const long long total = B.cfg_off[B.n_cfg];

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
    const StrRec* recs = B.rec + (long long)c * I.n_sec;
    lo = 0;
    hi = I.n_sec - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
    }
    const StrRec R = recs[lo];
    const int col0 = (local - R.loc_off) * kPanel;
    const int ncols = min(kPanel, R.width - col0);
    const long long base = B.offsets[c];
    const int n = (int)(B.offsets[c + 1] - base);
    const double* tau = B.tau + base;
    const int* ops = B.op + base;

    int s = R.q_start, pos = R.jstar;
    if (tid < kPanel) colexp[tid] = 0;
    {
      const int d = I.dim[s];
      const double dt = (n == 0) ? I.beta : dtp(tau, n, pos, I.beta);
      const double* e = I.esh + I.eoff[s];
      for (int r = tid; r < XR; r += NT) pa[r] = (r < d) ? exp(-dt * e[r]) : 0.0;
    }
    __syncthreads();

    PanelRes out;
    out.re = out.im = out.e2 = 0.0;
    if (n == 0) {
      if (tid == 0) {
        double sum = 0.0;
        for (int cc = 0; cc < ncols; ++cc) sum += pa[col0 + cc];
        out.re = sum;
      }
    } else {
      for (int t = 0; t < n - 1; ++t) {
        const int idx = s * I.nops + ops[pos];
        const int s2 = I.next[idx];
        const int d_in = I.dim[s], d_out = I.dim[s2];
        const int ld = (d_out + 15) & ~15;
        const int ntiles = ld >> 4;
        const double* Fr = I.pool + I.boff[idx];
        const double* Fi = Fr + (long long)ld * ((d_in + 3) & ~3);
        const int pos2 = (pos + 1 == n) ? 0 : pos + 1;
        {
          const double dt2 = dtp(tau, n, pos2, I.beta);
          const double* e = I.esh + I.eoff[s2];
          for (int r = tid; r < ld; r += NT) pb[r] = (r < d_out) ? exp(-dt2 * e[r]) : 0.0;
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
        s = s2;
        pos = pos2;
      }

      // last operator: only the diagonal of F * X (rows col0 .. col0+ncols)
      {
        const int idx = s * I.nops + ops[pos];
        const int s2 = I.next[idx];
        const int d_in = I.dim[s];
        const int ld = (I.dim[s2] + 15) & ~15;
        const double* Fr = I.pool + I.boff[idx];
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
  const int flags = B.cfg_flags[c];
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
      double sr = 0.0, si = 0.0;
      for (int q = 0; q < I.n_sec; ++q) {
        const StrRec R = recs[q];
        for (int p = 0; p < R.n_panels; ++p) {
          const PanelRes P = res[R.loc_off + p];
          if (P.re != 0.0 || P.im != 0.0) {
            const double f = exp(P.e2 * ln2 - R.L - lmax);
            sr += P.re * f;
            si += P.im * f;
          }
        }
      }
      v.re = sr;
      v.im = si;
      v.log_scale = lmax - I.beta * I.E0;
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
Variant make_variant() {
  return Variant{reinterpret_cast<const void*>(&k_chain<CPLX, NW, MAXT>), NW, MAXT, CPLX};
}

bool pick_variant(const DevImp& imp, Variant* v) {
  const int tiles = imp.xrows / 16;
  if (imp.is_complex) {
    if (tiles <= 8) *v = make_variant<true, 4, 2>();
    else if (tiles <= 16) *v = make_variant<true, 8, 2>();
    else if (tiles <= 32) *v = make_variant<true, 8, 4>();
    else if (tiles <= 64) *v = make_variant<true, 16, 4>();
    else return false;
  } else {
    if (tiles <= 8) *v = make_variant<false, 4, 2>();
    else if (tiles <= 16) *v = make_variant<false, 8, 2>();
    else if (tiles <= 32) *v = make_variant<false, 8, 4>();
    else if (tiles <= 64) *v = make_variant<false, 16, 4>();
    else return false;
  }
  return true;
}

constexpr size_t kMaxLds = 160 * 1024;

}  // namespace

size_t chain_lds_bytes(const DevImp& imp) {
  Variant v;
  if (!pick_variant(imp, &v)) return 0;
  const size_t doubles = v.cplx ? (v.nw == 4 ? chain_lds_doubles<true, 4>(imp.xrows)
                                  : v.nw == 8 ? chain_lds_doubles<true, 8>(imp.xrows)
                                              : chain_lds_doubles<true, 16>(imp.xrows))
                                : (v.nw == 4 ? chain_lds_doubles<false, 4>(imp.xrows)
                                  : v.nw == 8 ? chain_lds_doubles<false, 8>(imp.xrows)
                                              : chain_lds_doubles<false, 16>(imp.xrows));
  return doubles * sizeof(double);
}

int chain_max_rows(int is_complex) { return is_complex ? 576 : 1024; }

int chain_grid(const DevImp& imp, int device, size_t* lds_bytes) {
  Variant v;
  if (!pick_variant(imp, &v)) return 0;
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

hipError_t launch_chain(const DevImp& imp, const BatchArgs& b, int grid, hipStream_t stream) {
  Variant v;
  if (!pick_variant(imp, &v) || grid <= 0) return hipErrorInvalidValue;
  const size_t bytes = chain_lds_bytes(imp);
  void* args[] = {const_cast<DevImp*>(&imp), const_cast<BatchArgs*>(&b)};
  return hipLaunchKernel(v.fn, dim3(grid), dim3(v.nw * 64), args, bytes, stream);
}

}  // namespace ctr
