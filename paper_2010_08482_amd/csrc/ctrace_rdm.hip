// Density-matrix estimator of a batch (Sec. 2.3.2): for every configuration
// C with weight w(C) != 0,
//
//   R(C) = (beta w)^-1 int_0^beta A(tau) dtau,
//
// A(tau) the time-ordered product cut at tau and closed the other way round,
// block diagonal in the sectors; the output is sum_C weight_C R(C), one dense
// block per sector in that sector's eigenbasis.
//
// Per sector string s (rotated to start at its narrowest sector, width N) the
// cut product inside interval p (the gap in front of rotated operator p, in
// sector s_p) factorises through the N columns of the start sector:
//
//   A(tau) = [P(t) X_p] [Z_p P(D_p - t)],   t = time since the interval began,
//   X_p = F_{p-1} P_{p-1} ... F_0 P_0                (d(s_p) x N, columns k)
//   Z_p = F_{n-1} P_{n-1} ... P_{p+1} F_p            (N x d(s_p), rows k)
//
// so its integral over the interval is sum_k X_p[u][k] Z_p[k][v] K(E_u, E_v, D_p)
// with K(a, b, D) = int_0^D e^{-t a} e^{-(D-t) b} dt in closed form.  The trace
// of every cut product is the string's weight, hence Tr R = 1.
//
//   k_rdm  persistent, one workgroup per (string, panel of 16 columns k): the
//          forward chain X_p is kept for every p (per-workgroup global
//          buffer, per-column powers of two), then the backward chain Z_p runs
//          from p = n-1 down to 0 and adds each interval's contribution to the
//          sector's block with atomic FP64 adds.  FP64 VALU products: the
//          estimator is sampled next to the trace, not in its hot loop.
#include <math.h>

#include "ctrace_internal.h"

namespace ctr {

namespace {

__device__ __forceinline__ double gap_in_front(const double* tau, int n, int p, double beta) {
  return p ? tau[p] - tau[p - 1] : tau[0] + beta - tau[n - 1];
}

// int_0^D exp(-t a) exp(-(D - t) b) dt
__device__ __forceinline__ double interval_kernel(double a, double b, double D) {
  const double d = a - b;
  if (fabs(d) <= 1e-12 * fmax(1.0, fmax(fabs(a), fabs(b)))) return D * exp(-D * 0.5 * (a + b));
  return (exp(-D * b) - exp(-D * a)) / d;
}

constexpr int kRdmThreads = 256;
constexpr int kRdmCols = kPanel;  // 16 columns k per work item

}  // namespace

__global__ __launch_bounds__(kRdmThreads) void k_rdm(DevImp I, BatchArgs B, RdmArgs D) {
  __shared__ long long s_w;
  __shared__ double s_dt[kMaxOps];
  __shared__ short s_op[kMaxOps];
  __shared__ short s_path[kMaxOps + 1];
  __shared__ int s_exf[kRdmCols];
  __shared__ int s_exz[kRdmCols];
  __shared__ double s_red[kRdmThreads];
  __shared__ double s_fr[kRdmCols], s_fi[kRdmCols];
  __shared__ double s_prop[kRdmMaxRows];
  const int tid = threadIdx.x;
  const int XR = I.xrows;
  const int PL = I.is_complex ? 2 : 1;
  const size_t colsz = (size_t)XR * kRdmCols;  // one plane of one stored X_p (rows x 16)
  // this workgroup's buffers: X_0 .. X_{slots-1} (PL planes each), Z ping-pong, exponents of every X_p
  double* Xs = D.buf + (size_t)blockIdx.x * D.per_wg;
  double* Zb[2] = {Xs + (size_t)D.slots * PL * colsz, Xs + (size_t)(D.slots + 1) * PL * colsz};
  int* exs = (int*)(Zb[1] + PL * colsz);  // [slots * 16]
  const long long total = B.cfg_off[B.n_cfg];
  const double ln2 = 0.69314718055994530942;
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
    const StrRec* recs = B.rec + (long long)c * I.n_sec;
    lo = 0;
    hi = I.n_sec - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
    }
    const StrRec R = recs[lo];
    const int col0 = (local - R.loc_off) * kRdmCols;
    const int nc = min(kRdmCols, R.width - col0);
    const long long base = B.offsets[c];
    const int n = (int)(B.offsets[c + 1] - base);
    const double wre = D.w[2 * c], wim = D.w[2 * c + 1], wlog = D.wlog[c];
    if (wre == 0.0 && wim == 0.0) {  // zero (or rejected) trace: no estimator
      __syncthreads();
      continue;
    }
    // coefficient of every contribution: weight / (beta w), the powers of two and exp(-L) come per column
    const double den = wre * wre + wim * wim;
    const double cre0 = (D.weight[2 * c] * wre + D.weight[2 * c + 1] * wim) / (den * I.beta);
    const double cim0 = (D.weight[2 * c + 1] * wre - D.weight[2 * c] * wim) / (den * I.beta);
    const int nn = n > 0 ? n : 1;  // order zero: one interval of length beta in the start sector
    for (int t = tid; t < nn; t += kRdmThreads) {
      if (n > 0) {
        const int p = (R.jstar + t) % n;
        s_op[t] = (short)B.op[base + p];
        s_dt[t] = gap_in_front(B.tau + base, n, p, I.beta);
      } else {
        s_op[t] = -1;
        s_dt[t] = I.beta;
      }
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
    // X_0 = the panel's columns of the identity
    {
      const int d0 = I.dim[R.q_start];
      for (int i = tid; i < d0 * kRdmCols; i += kRdmThreads) {
        const int m = i / kRdmCols, cc = i % kRdmCols;
        Xs[(size_t)m * kRdmCols + cc] = (cc < nc && m == col0 + cc) ? 1.0 : 0.0;
        if (PL == 2) Xs[colsz + (size_t)m * kRdmCols + cc] = 0.0;
      }
      if (tid < kRdmCols) exs[tid] = 0;
    }
    __syncthreads();
    // forward: X_{p+1} = F_p P(dt_p) X_p, rescaled per column
    for (int p = 0; p < n - 1; ++p) {
      const int s = s_path[p], s2 = s_path[p + 1];
      const int d_in = I.dim[s], d_out = I.dim[s2];
      const int ld = (d_out + 15) & ~15, kp = (d_in + 3) & ~3;
      const double* Fr = I.pool + I.boff[s * I.nops + s_op[p]];
      const double* Fi = Fr + (size_t)ld * kp;
      const double* e = I.esh + I.eoff[s];
      const double dt = s_dt[p];
      const double* Xr = Xs + (size_t)p * PL * colsz;
      double* Yr = Xs + (size_t)(p + 1) * PL * colsz;
      for (int k = tid; k < d_in; k += kRdmThreads) s_prop[k] = exp(-dt * e[k]);
      __syncthreads();
      for (int i = tid; i < d_out * kRdmCols; i += kRdmThreads) {
        const int m = i / kRdmCols, cc = i % kRdmCols;
        double ar = 0.0, ai = 0.0;
        for (int k = 0; k < d_in; ++k) {
          const double pk = s_prop[k];
          const double fr = Fr[(size_t)k * ld + m], xr = Xr[(size_t)k * kRdmCols + cc] * pk;
          if (PL == 2) {
            const double fi = Fi[(size_t)k * ld + m], xi = Xr[colsz + (size_t)k * kRdmCols + cc] * pk;
            ar += fr * xr - fi * xi;
            ai += fr * xi + fi * xr;
          } else {
            ar += fr * xr;
          }
        }
        Yr[(size_t)m * kRdmCols + cc] = ar;
        if (PL == 2) Yr[colsz + (size_t)m * kRdmCols + cc] = ai;
      }
      __syncthreads();
      // per-column maximum, then the exact power-of-two rescale
      for (int cc = 0; cc < kRdmCols; ++cc) {
        double mx = 0.0;
        for (int m = tid; m < d_out; m += kRdmThreads) {
          mx = fmax(mx, fabs(Yr[(size_t)m * kRdmCols + cc]));
          if (PL == 2) mx = fmax(mx, fabs(Yr[colsz + (size_t)m * kRdmCols + cc]));
        }
        s_red[tid] = mx;
        __syncthreads();
        for (int off = kRdmThreads / 2; off > 0; off >>= 1) {
          if (tid < off) s_red[tid] = fmax(s_red[tid], s_red[tid + off]);
          __syncthreads();
        }
        if (tid == 0) {
          int ex = 0;
          if (s_red[0] > 0.0) frexp(s_red[0], &ex);
          s_exf[cc] = ex;
        }
        __syncthreads();
      }
      for (int i = tid; i < d_out * kRdmCols; i += kRdmThreads) {
        const int m = i / kRdmCols, cc = i % kRdmCols;
        const double sc = ldexp(1.0, -s_exf[cc]);
        Yr[(size_t)m * kRdmCols + cc] *= sc;
        if (PL == 2) Yr[colsz + (size_t)m * kRdmCols + cc] *= sc;
      }
      if (tid < kRdmCols) exs[(p + 1) * kRdmCols + tid] = exs[p * kRdmCols + tid] + s_exf[tid];
      __syncthreads();
    }
    // backward: Z_{n-1} = rows col0.. of F_{n-1} (order zero: the identity rows); Z_p = (Z_{p+1} P_{p+1}) F_p
    int zc = 0;
    for (int p = nn - 1; p >= 0; --p) {
      const int s = s_path[p];
      const int d = I.dim[s];
      double* Z = Zb[zc];
      if (p == nn - 1) {
        if (n > 0) {
          const int s2 = s_path[n];  // = the start sector
          const int ld = (I.dim[s2] + 15) & ~15, kp = (d + 3) & ~3;
          const double* Fr = I.pool + I.boff[s * I.nops + s_op[p]];
          const double* Fi = Fr + (size_t)ld * kp;
          for (int i = tid; i < d * kRdmCols; i += kRdmThreads) {
            const int v = i / kRdmCols, cc = i % kRdmCols;
            Z[(size_t)v * kRdmCols + cc] = cc < nc ? Fr[(size_t)v * ld + col0 + cc] : 0.0;
            if (PL == 2) Z[colsz + (size_t)v * kRdmCols + cc] = cc < nc ? Fi[(size_t)v * ld + col0 + cc] : 0.0;
          }
        } else {
          for (int i = tid; i < d * kRdmCols; i += kRdmThreads) {
            const int v = i / kRdmCols, cc = i % kRdmCols;
            Z[(size_t)v * kRdmCols + cc] = (cc < nc && v == col0 + cc) ? 1.0 : 0.0;
            if (PL == 2) Z[colsz + (size_t)v * kRdmCols + cc] = 0.0;
          }
        }
        if (tid < kRdmCols) s_exz[tid] = 0;
      } else {
        // Z_p[k][v] = sum_m Z_{p+1}[k][m] e^{-dt_{p+1} E_m} F_p[m][v], stored as [v][k]
        const int s2 = s_path[p + 1];
        const int d2 = I.dim[s2];
        const int ld = (d2 + 15) & ~15, kp = (d + 3) & ~3;
        const double* Fr = I.pool + I.boff[s * I.nops + s_op[p]];
        const double* Fi = Fr + (size_t)ld * kp;
        const double* e2 = I.esh + I.eoff[s2];
        const double dt2 = s_dt[p + 1];
        const double* Zn = Zb[zc ^ 1];
        for (int m = tid; m < d2; m += kRdmThreads) s_prop[m] = exp(-dt2 * e2[m]);
        __syncthreads();
        for (int i = tid; i < d * kRdmCols; i += kRdmThreads) {
          const int v = i / kRdmCols, cc = i % kRdmCols;
          double ar = 0.0, ai = 0.0;
          for (int m = 0; m < d2; ++m) {
            const double pm = s_prop[m];
            const double fr = Fr[(size_t)v * ld + m], zr = Zn[(size_t)m * kRdmCols + cc] * pm;
            if (PL == 2) {
              const double fi = Fi[(size_t)v * ld + m], zi = Zn[colsz + (size_t)m * kRdmCols + cc] * pm;
              ar += zr * fr - zi * fi;
              ai += zr * fi + zi * fr;
            } else {
              ar += zr * fr;
            }
          }
          Z[(size_t)v * kRdmCols + cc] = ar;
          if (PL == 2) Z[colsz + (size_t)v * kRdmCols + cc] = ai;
        }
        __syncthreads();
        for (int cc = 0; cc < kRdmCols; ++cc) {
          double mx = 0.0;
          for (int v = tid; v < d; v += kRdmThreads) {
            mx = fmax(mx, fabs(Z[(size_t)v * kRdmCols + cc]));
            if (PL == 2) mx = fmax(mx, fabs(Z[colsz + (size_t)v * kRdmCols + cc]));
          }
          s_red[tid] = mx;
          __syncthreads();
          for (int off = kRdmThreads / 2; off > 0; off >>= 1) {
            if (tid < off) s_red[tid] = fmax(s_red[tid], s_red[tid + off]);
            __syncthreads();
          }
          if (tid == 0) {
            int ex = 0;
            if (s_red[0] > 0.0) frexp(s_red[0], &ex);
            s_exf[cc] = ex;
          }
          __syncthreads();
        }
        for (int i = tid; i < d * kRdmCols; i += kRdmThreads) {
          const int v = i / kRdmCols, cc = i % kRdmCols;
          const double sc = ldexp(1.0, -s_exf[cc]);
          Z[(size_t)v * kRdmCols + cc] *= sc;
          if (PL == 2) Z[colsz + (size_t)v * kRdmCols + cc] *= sc;
        }
        if (tid < kRdmCols) s_exz[tid] += s_exf[tid];
      }
      __syncthreads();
      // factor of column k: coefficient x 2^(exponents of X_p and Z_p) x exp(-L) relative to w
      if (tid < kRdmCols) {
        double f = 0.0;
        if (tid < nc) {
          const double lg = (exs[p * kRdmCols + tid] + s_exz[tid]) * ln2 - R.L - wlog;
          f = exp(lg);
        }
        s_fr[tid] = f * cre0;
        s_fi[tid] = f * cim0;
      }
      __syncthreads();
      // interval p: rho(s)[u][v] += sum_k X_p[u][k] Z_p[k][v] K(E_u, E_v, dt_p) f_k
      {
        const double* Xp = Xs + (size_t)p * PL * colsz;
        const double* e = I.esh + I.eoff[s];
        const double dt = s_dt[p];
        double* rho = D.rho + 2 * D.rho_off[s];
        for (int i = tid; i < d * d; i += kRdmThreads) {
          const int u = i / d, v = i % d;
          double sr = 0.0, si = 0.0;
          for (int cc = 0; cc < nc; ++cc) {
            const double xr = Xp[(size_t)u * kRdmCols + cc], zr = Z[(size_t)v * kRdmCols + cc];
            double pr = xr * zr, pi = 0.0;
            if (PL == 2) {
              const double xi = Xp[colsz + (size_t)u * kRdmCols + cc], zi = Z[colsz + (size_t)v * kRdmCols + cc];
              pr -= xi * zi;
              pi = xr * zi + xi * zr;
            }
            sr += pr * s_fr[cc] - pi * s_fi[cc];
            si += pr * s_fi[cc] + pi * s_fr[cc];
          }
          if (sr != 0.0 || si != 0.0) {
            const double k = interval_kernel(e[u], e[v], dt);
            atomicAdd(rho + 2 * (size_t)i, sr * k);
            atomicAdd(rho + 2 * (size_t)i + 1, si * k);
          }
        }
      }
      zc ^= 1;
      __syncthreads();
    }
  }
}

size_t rdm_buffer_doubles(const DevImp& imp, int slots) {
  const size_t PL = imp.is_complex ? 2 : 1;
  const size_t colsz = (size_t)imp.xrows * kRdmCols;
  // X_0 .. X_{slots-1}, two Z buffers, the per-position column exponents (ints), 256-byte aligned
  const size_t n = (size_t)(slots + 2) * PL * colsz + ((size_t)slots * kRdmCols + 1) / 2;
  return (n + 31) & ~(size_t)31;
}

int rdm_grid(int device) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  return cus;
}

hipError_t launch_rdm(const DevImp& imp, const BatchArgs& b, const RdmArgs& d, int grid, hipStream_t stream) {
  if (grid <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rdm, dim3(grid), dim3(kRdmThreads), 0, stream, imp, b, d);
  return hipGetLastError();
}

}  // namespace ctr
