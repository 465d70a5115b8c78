// Block-grouped evaluation of a batch of traces (gfx950).
//
// Every surviving sector string (Sec. 3.3.1) is a chain X <- F_op(q) P X over
// its start sector's columns.  Strings are independent, so instead of running
// each string's whole chain alone (re-reading each operator block once per
// string), all strings of the batch advance one operator per round, and in
// every round the strings standing at the same block F_op(q) are grouped:
// their columns are packed side by side and multiplied by F in one wide
// FP64 MFMA product, so each block is read once per 32 or 64 columns.
//
//   k_gstrings  one thread per surviving string: configuration and record
//   k_gscan1    one workgroup: column offsets of the strings (exclusive scan
//               of their widths), total columns, number of rounds
//   k_gwalk     one thread per string: walks its rotated sector path and
//               counts, per (round, block), strings and columns
//   k_gsched    one workgroup per round: group offsets and work items
//   k_gwalk     (again) one thread per string: its position in every round's groups
//   k_gcolpref  one workgroup per round: column offsets in group order
//   k_gscan2    one workgroup: offsets of every round's columns and items
//   k_gkeys     one thread per (round, group): the group of every work item
//   k_gitems    one thread per (round, string): global column and gap of
//               every column-step, in group order (work items read them
//               with one coalesced load instead of searching)
//   k_gfirst    one workgroup per string: the first operator (a column-scaled
//               copy of F, the carried matrix starts as the identity)
//   k_gstep     persistent, one launch per round: work items of 64 (real) or
//               32 (complex) columns of one group, F * X on FP64 MFMA 16x16x4
//               with the propagator of the next gap and the per-column
//               power-of-two rescale fused into the epilogue; strings at
//               their last operator only form the diagonal of F * X
//   k_gstep_wave  the same for sectors of at most 128 (real) or 32 (complex)
//               states: one wavefront per item of 16 or 32 columns, no barriers
//   k_gcombine  one wavefront per configuration: (mantissa, exponent) merge
//               of all columns of all its strings
#include <math.h>

#include "ctrace_internal.h"

namespace ctr {

namespace {

__device__ __forceinline__ double gap_before(const double* tau, int n, int p, double beta) {
  // imaginary-time gap in front of operator p; position 0 carries the wrap gap
  return p ? tau[p] - tau[p - 1] : tau[0] + beta - tau[n - 1];
}

// Largest i in [lo, hi) with a[i] <= x (a non-decreasing, a[lo] <= x).
template <typename T>
__device__ __forceinline__ int last_le(const T* a, int lo, int hi, T x) {
  hi -= 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Block-wide exclusive scan of v over the calling workgroup (blockDim.x
// threads, at most 1024); returns the exclusive prefix, *total the sum.
template <typename T>
__device__ T block_exclusive_scan(T v, T* s_tmp, T* total) {
  const int t = threadIdx.x, nt = blockDim.x;
  s_tmp[t] = v;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {
    const T u = (t >= off) ? s_tmp[t - off] : T(0);
    __syncthreads();
    s_tmp[t] += u;
    __syncthreads();
  }
  const T incl = s_tmp[t];
  *total = s_tmp[nt - 1];
  __syncthreads();
  return incl - v;
}

}  // namespace

// ---------------------------------------------------------------------------
// strings of the batch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gstrings(DevImp I, BatchArgs B, GroupArgs G) {
  const long long w = (long long)blockIdx.x * 256 + threadIdx.x;
  const long long S = B.cfg_off[B.n_cfg];
  if (w >= S) return;
  const int c = last_le<long long>(B.cfg_off, 0, B.n_cfg, w);
  const int local = (int)(w - B.cfg_off[c]);
  const StrRec* recs = B.rec + (long long)c * I.n_sec;
  int lo = 0, hi = I.n_sec - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (recs[mid].loc_off <= local) lo = mid; else hi = mid - 1;
  }
  G.s_cfg[w] = c;
  G.s_rec[w] = lo;
  G.s_width[w] = recs[lo].width;
  G.s_n[w] = (int)(B.offsets[c + 1] - B.offsets[c]);
}

__global__ __launch_bounds__(1024) void k_gscan1(DevImp I, BatchArgs B, GroupArgs G) {
  __shared__ long long s_tmp[1024];
  __shared__ long long s_cs[1024], s_ns[1024];
  __shared__ int s_max[1024];
  const int t = threadIdx.x;
  const long long S = B.cfg_off[B.n_cfg];
  const long long chunk = (S + 1023) / 1024;
  const long long lo = min((long long)t * chunk, S), hi = min(lo + chunk, S);
  long long sum = 0, cs = 0, ns = 0;
  int nmax = 0;
  for (long long w = lo; w < hi; ++w) {
    const int wd = G.s_width[w], n = G.s_n[w];
    sum += wd;
    cs += (long long)wd * max(n - 1, 0);
    ns += max(n - 1, 0);
    nmax = max(nmax, n);
  }
  long long total = 0;
  long long run = block_exclusive_scan<long long>(sum, s_tmp, &total);
  for (long long w = lo; w < hi; ++w) {
    G.s_colbase[w] = run;
    run += G.s_width[w];
  }
  s_max[t] = nmax;
  s_cs[t] = cs;
  s_ns[t] = ns;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) {
      s_max[t] = max(s_max[t], s_max[t + off]);
      s_cs[t] += s_cs[t + off];
      s_ns[t] += s_ns[t + off];
    }
    __syncthreads();
  }
  if (t == 0) {
    G.info[0] = S;
    G.info[1] = total;
    G.info[2] = s_max[0];  // rounds: the close of a string of n operators is round n - 1
    G.info[3] = s_cs[0];
    // work items: at most one partial item per (round, group) on top of the full ones, times the
    // row chunks of the largest block
    const long long nrc = G.rchunk > 0 ? (I.xrows + G.rchunk - 1) / G.rchunk : 1;
    G.info[4] = (s_cs[0] / min(G.cw_step, G.cw_close) + s_ns[0] + 1) * nrc;
  }
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
// Group key of a string at round r >= 1: the block it applies, offset by NB
// at its last operator (the close).
__global__ __launch_bounds__(256) void k_gwalk(DevImp I, BatchArgs B, GroupArgs G, int scatter) {
  const long long w = (long long)blockIdx.x * 256 + threadIdx.x;
  if (w >= G.S) return;
  const int c = G.s_cfg[w];
  const StrRec R = B.rec[(long long)c * I.n_sec + G.s_rec[w]];
  const long long base = B.offsets[c];
  const int n = (int)(B.offsets[c + 1] - base);
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  int cur = R.q_start;
  for (int r = 0; r < n; ++r) {
    const int op = B.op[base + (R.jstar + r) % n];
    const int blk = cur * I.nops + op;
    if (r >= 1) {
      const int key = (r < n - 1) ? blk : NB + blk;
      const long long rk = (long long)r * NK + key;
      if (!scatter) {
        atomicAdd(G.hist + rk, 1);
        atomicAdd(G.hcols + rk, R.width);
      } else {
        const int pos = G.gstart[(long long)r * (NK + 1) + key] + atomicAdd(G.cursor + rk, 1);
        G.sorted[(long long)r * G.S + pos] = (int)w;
      }
    }
    cur = I.next[blk];
  }
}

__global__ __launch_bounds__(1024) void k_gsched(DevImp I, GroupArgs G) {
  __shared__ int s_tmp[1024];
  const int r = blockIdx.x + 1;
  if (r >= G.R) return;
  const int t = threadIdx.x;
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  const int chunk = (NK + 1023) / 1024;
  const int lo = min(t * chunk, NK), hi = min(lo + chunk, NK);
  const int* hist = G.hist + (long long)r * NK;
  const int* hcols = G.hcols + (long long)r * NK;
  int* gstart = G.gstart + (long long)r * (NK + 1);
  int* istart = G.istart + (long long)r * (NK + 1);
  // items of group k: column tiles, times the row chunks of its block for products
  auto items = [&](int k) {
    const int cw = k < NB ? G.cw_step : G.cw_close;
    int n = (hcols[k] + cw - 1) / cw;
    if (k < NB && G.rchunk > 0 && n > 0) n *= (I.dim[I.next[k]] + G.rchunk - 1) / G.rchunk;
    return n;
  };
  int s1 = 0, s2 = 0;
  for (int k = lo; k < hi; ++k) {
    s1 += hist[k];
    s2 += items(k);
  }
  int tot1 = 0, tot2 = 0;
  int run1 = block_exclusive_scan<int>(s1, s_tmp, &tot1);
  int run2 = block_exclusive_scan<int>(s2, s_tmp, &tot2);
  for (int k = lo; k < hi; ++k) {
    gstart[k] = run1;
    istart[k] = run2;
    run1 += hist[k];
    run2 += items(k);
  }
  if (t == 0) {
    gstart[NK] = tot1;
    istart[NK] = tot2;
    G.n_items[r] = tot2;
  }
}

__global__ __launch_bounds__(1024) void k_gcolpref(DevImp I, BatchArgs B, GroupArgs G) {
  __shared__ int s_tmp[1024];
  const int r = blockIdx.x + 1;
  if (r >= G.R) return;
  const int t = threadIdx.x;
  const int NK = 2 * I.n_sec * I.nops;
  const int cnt = G.gstart[(long long)r * (NK + 1) + NK];
  const int chunk = (cnt + 1023) / 1024;
  const int lo = min(t * chunk, cnt), hi = min(lo + chunk, cnt);
  const int* sorted = G.sorted + (long long)r * G.S;
  int* colpref = G.colpref + (long long)r * G.S;
  int sum = 0;
  for (int p = lo; p < hi; ++p) sum += G.s_width[sorted[p]];
  int tot = 0;
  int run = block_exclusive_scan<int>(sum, s_tmp, &tot);
  for (int p = lo; p < hi; ++p) {
    colpref[p] = run;
    run += G.s_width[sorted[p]];
  }
  if (t == 0) G.rcols[r] = tot;
}

// Offsets of every round's column-steps and work items (rounds 1 .. R-1).
__global__ __launch_bounds__(1024) void k_gscan2(GroupArgs G) {
  __shared__ long long s_tmp[1024];
  const int t = threadIdx.x;
  const int chunk = (G.R + 1023) / 1024;
  const int lo = min(t * chunk, G.R), hi = min(lo + chunk, G.R);
  long long c = 0, it = 0;
  for (int r = lo; r < hi; ++r) {
    c += r >= 1 ? G.rcols[r] : 0;
    it += r >= 1 ? G.n_items[r] : 0;
  }
  long long tot = 0;
  long long rc = block_exclusive_scan<long long>(c, s_tmp, &tot);
  long long ri = block_exclusive_scan<long long>(it, s_tmp, &tot);
  for (int r = lo; r < hi; ++r) {
    G.rcoloff[r] = rc;
    G.ritemoff[r] = ri;
    rc += r >= 1 ? G.rcols[r] : 0;
    ri += r >= 1 ? G.n_items[r] : 0;
  }
}

// Group of every work item of round r.
__global__ __launch_bounds__(256) void k_gkeys(DevImp I, GroupArgs G) {
  const int NK = 2 * I.n_sec * I.nops;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)(G.R - 1) * NK) return;
  const int r = (int)(idx / NK) + 1, key = (int)(idx % NK);
  const int* istart = G.istart + (long long)r * (NK + 1);
  int* out = G.item_key + G.ritemoff[r];
  for (int it = istart[key]; it < istart[key + 1]; ++it) out[it] = key;
}

// Column-steps of round r in group order: global column and the gap in front
// of the string's next operator (or, at its last operator, the column's index
// in the start sector, where the diagonal is taken).
__global__ __launch_bounds__(256) void k_gitems(DevImp I, BatchArgs B, GroupArgs G) {
  const int NK = 2 * I.n_sec * I.nops;
  const long long idx = (long long)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (long long)(G.R - 1) * G.S) return;
  const int r = (int)(idx / G.S) + 1;
  const int p = (int)(idx % G.S);
  if (p >= G.gstart[(long long)r * (NK + 1) + NK]) return;
  const int w = G.sorted[(long long)r * G.S + p];
  const int n = G.s_n[w], width = G.s_width[w];
  const long long cb = G.s_colbase[w];
  const long long base = G.rcoloff[r] + G.colpref[(long long)r * G.S + p];
  if (r == n - 1) {
    for (int j = 0; j < width; ++j) {
      G.colg[base + j] = (int)(cb + j);
      G.colaux[base + j] = (double)j;
    }
  } else {
    const int c = G.s_cfg[w];
    const StrRec R = B.rec[(long long)c * I.n_sec + G.s_rec[w]];
    const long long o = B.offsets[c];
    const double dt = gap_before(B.tau + o, n, (R.jstar + r + 1) % n, I.beta);
    for (int j = 0; j < width; ++j) {
      G.colg[base + j] = (int)(cb + j);
      G.colaux[base + j] = dt;
    }
  }
}

// ---------------------------------------------------------------------------
// round 0: the first operator of every string
// ---------------------------------------------------------------------------
template <bool CPLX>
__global__ __launch_bounds__(256) void k_gfirst(DevImp I, BatchArgs B, GroupArgs G) {
  const long long w = blockIdx.x;
  if (w >= G.S) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = G.s_cfg[w];
  const StrRec R = B.rec[(long long)c * I.n_sec + G.s_rec[w]];
  const long long base = B.offsets[c];
  const int n = (int)(B.offsets[c + 1] - base);
  const long long cb = G.s_colbase[w];
  const int s = R.q_start;
  const double* e_s = I.esh + I.eoff[s];
  if (n == 0) {
    // partition-function string: trace of the diagonal propagator
    for (int j = threadIdx.x; j < R.width; j += 256) {
      PanelRes o;
      o.re = exp(-I.beta * e_s[j]);
      o.im = 0.0;
      o.e2 = 0.0;
      G.colres[cb + j] = o;
    }
    return;
  }
  const double* tau = B.tau + base;
  const int op0 = B.op[base + R.jstar];
  const int blk = s * I.nops + op0;
  const int s2 = I.next[blk];
  const int d_out = I.dim[s2];
  const int ld = (d_out + 15) & ~15;
  const double* Fr = I.pool + I.boff[blk];
  const double* Fi = Fr + (long long)ld * ((I.dim[s] + 3) & ~3);
  const double dt0 = gap_before(tau, n, R.jstar, I.beta);
  const double dt1 = gap_before(tau, n, (R.jstar + 1) % n, I.beta);
  const double* e_2 = I.esh + I.eoff[s2];
  const long long plane = G.T * (long long)I.xrows;
  double* X = G.X[0];
  for (int j = wave; j < R.width; j += 4) {
    const double p0 = exp(-dt0 * e_s[j]);
    double vr[8], vi[8];
    double cm = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = lane + 64 * u;
      vr[u] = vi[u] = 0.0;
      if (m < d_out) {
        const double p = p0 * exp(-dt1 * e_2[m]);
        vr[u] = Fr[(long long)j * ld + m] * p;
        cm = fmax(cm, fabs(vr[u]));
        if (CPLX) {
          vi[u] = Fi[(long long)j * ld + m] * p;
          cm = fmax(cm, fabs(vi[u]));
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) cm = fmax(cm, __shfl_xor(cm, off));
    int e = 0;
    if (cm > 0.0) frexp(cm, &e);
    const double sc = ldexp(1.0, -e);
    double* col = X + (cb + j) * I.xrows;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = lane + 64 * u;
      if (m < ld) {
        col[m] = vr[u] * sc;
        if (CPLX) col[plane + m] = vi[u] * sc;
      }
    }
    if (lane == 0) G.colexp[cb + j] = e;
  }
}

// Round 0 for sectors of any size (row-chunked rounds): the column-scaled
// copy of F is stored unscaled; its power of two is left pending for round 1.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_gfirst_big(DevImp I, BatchArgs B, GroupArgs G) {
  const long long w = blockIdx.x;
  if (w >= G.S) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = G.s_cfg[w];
  const StrRec R = B.rec[(long long)c * I.n_sec + G.s_rec[w]];
  const long long base = B.offsets[c];
  const int n = (int)(B.offsets[c + 1] - base);
  const long long cb = G.s_colbase[w];
  const int s = R.q_start;
  const double* e_s = I.esh + I.eoff[s];
  if (n == 0) {
    for (int j = threadIdx.x; j < R.width; j += 256) {
      PanelRes o;
      o.re = exp(-I.beta * e_s[j]);
      o.im = 0.0;
      o.e2 = 0.0;
      G.colres[cb + j] = o;
    }
    return;
  }
  const double* tau = B.tau + base;
  const int blk = s * I.nops + B.op[base + R.jstar];
  const int s2 = I.next[blk];
  const int d_out = I.dim[s2];
  const int ld = (d_out + 15) & ~15;
  const double* Fr = I.pool + I.boff[blk];
  const double* Fi = Fr + (long long)ld * ((I.dim[s] + 3) & ~3);
  const double dt0 = gap_before(tau, n, R.jstar, I.beta);
  const double dt1 = gap_before(tau, n, (R.jstar + 1) % n, I.beta);
  const double* e_2 = I.esh + I.eoff[s2];
  const long long plane = G.T * (long long)I.xrows;
  double* X = G.X[0];
  for (int j = wave; j < R.width; j += 4) {
    const double p0 = exp(-dt0 * e_s[j]);
    double* col = X + (cb + j) * I.xrows;
    double cm = 0.0;
    for (int m = lane; m < ld; m += 64) {
      const double p = m < d_out ? p0 * exp(-dt1 * e_2[m]) : 0.0;
      const double vr = Fr[(long long)j * ld + m] * p;
      col[m] = vr;
      cm = fmax(cm, fabs(vr));
      if (CPLX) {
        const double vi = Fi[(long long)j * ld + m] * p;
        col[plane + m] = vi;
        cm = fmax(cm, fabs(vi));
      }
    }
    for (int off = 32; off > 0; off >>= 1) cm = fmax(cm, __shfl_xor(cm, off));
    int e = 0;
    if (cm > 0.0) frexp(cm, &e);
    if (lane == 0) {
      G.colexp[cb + j] = 0;
      G.epend[1 * G.T + cb + j] = cm > 0.0 ? e : kNoExp;
      G.epend[2 * G.T + cb + j] = kNoExp;
    }
  }
}

// ---------------------------------------------------------------------------
// rounds r >= 1
// ---------------------------------------------------------------------------
template <bool CPLX, int NW, int RT, int CT>
__global__ __launch_bounds__(NW * 64) void k_gstep(DevImp I, BatchArgs B, GroupArgs G, int r) {
  constexpr int CW = CT * 16;            // columns per work item
  constexpr int NT = NW * 64;
  constexpr int KC = 64;                 // rows of X staged in LDS per chunk
  constexpr int LDB = KC + 1;            // odd stride: the 16 columns of a B fragment hit distinct banks
  constexpr int PL = CPLX ? 2 : 1;
  __shared__ double sB[2 * PL * CW * LDB];  // two staging buffers: chunk c in buffer c % 2
  __shared__ double s_cmax[NW * CW];
  __shared__ double s_dt[CW];
  __shared__ long long s_gcol[CW];
  __shared__ int s_e[CW];
  __shared__ int s_item;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ln = lane & 15, lq = lane >> 4;
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  const int XR = I.xrows;
  const long long plane = G.T * (long long)XR;
  const double* Xin = G.X[(r + 1) & 1];
  double* Xout = G.X[r & 1];
  const int* istart = G.istart + (long long)r * (NK + 1);
  const int* gstart = G.gstart + (long long)r * (NK + 1);
  const int* hcols = G.hcols + (long long)r * NK;
  const int* colpref = G.colpref + (long long)r * G.S;

  const long long* ritemoff = G.ritemoff;
  // item i is served by counter i % kGroupCounters
  const int n_items = G.n_items[r];
  const int slot = blockIdx.x % kGroupCounters;
  unsigned int* counter = G.counters + ((long long)r * kGroupCounters + slot) * 32;
  for (;;) {
    if (tid == 0) s_item = slot + kGroupCounters * (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= n_items) break;
    // group and column range of this item
    const int key = G.item_key[ritemoff[r] + item];
    const bool close = key >= NB;
    const int blk = close ? key - NB : key;
    const int cw = close ? G.cw_close : CW;
    const int c0 = (item - istart[key]) * cw;
    const int ncol = min(cw, hcols[key] - c0);
    const long long relbase = G.rcoloff[r] + colpref[gstart[key]] + c0;
    const int s = blk / I.nops;
    const int s2 = I.next[blk];
    const int d_in = I.dim[s], d_out = I.dim[s2];
    const int ld = (d_out + 15) & ~15;
    const int kp = (d_in + 3) & ~3;
    const double* Fr = I.pool + I.boff[blk];
    const double* Fi = Fr + (long long)ld * kp;

    if (close) {
      // diagonal of F * X: column j of the string meets row j of F
      for (int j = wave; j < ncol; j += NW) {
        const long long gcol = G.colg[relbase + j];
        const int jj = (int)G.colaux[relbase + j];
        const double* xr = Xin + gcol * XR;
        double sr = 0.0, si = 0.0;
        for (int k = lane; k < d_in; k += 64) {
          const double fr = Fr[(long long)k * ld + jj], x = xr[k];
          if (CPLX) {
            const double fi = Fi[(long long)k * ld + jj], xi = xr[plane + k];
            sr += fr * x - fi * xi;
            si += fr * xi + fi * x;
          } else {
            sr += fr * x;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        if (lane == 0) {
          PanelRes o;
          o.re = sr;
          o.im = si;
          o.e2 = (double)G.colexp[gcol];
          G.colres[gcol] = o;
        }
      }
      __syncthreads();
      continue;
    }

    // columns of this item: global column, next gap
    if (tid < CW) {
      s_gcol[tid] = tid < ncol ? (long long)G.colg[relbase + tid] : -1;
      s_dt[tid] = tid < ncol ? G.colaux[relbase + tid] : 0.0;
    }

    typedef double dbl4 __attribute__((ext_vector_type(4)));
    dbl4 acc_r[RT][CT], acc_i[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        acc_r[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
        acc_i[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
    const int ntiles = ld >> 4;
    // A fragments run kPD k-steps ahead of the products (a ring of kPD slots;
    // kPD divides the 16 k-steps of a staged chunk, so step s sits in slot s % kPD)
    constexpr int kPD = 2;
    double rr[kPD][RT], ri[kPD][RT];
#pragma unroll
    for (int d = 0; d < kPD; ++d)
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = wave + i * NW;
        rr[d][i] = ri[d][i] = 0.0;
        if (tile < ntiles && 4 * d < kp) {
          const long long a = (long long)(4 * d + lq) * ld + tile * 16 + ln;
          rr[d][i] = Fr[a];
          if (CPLX) ri[d][i] = Fi[a];
        }
      }
    for (int k0 = 0; k0 < kp; k0 += KC) {
      const int kc = min(KC, kp - k0);
      // one barrier per chunk after the first: the buffer written here was last
      // read two chunks ago, which every wavefront finished before the barrier
      // of the chunk in between
      double* sBc = sB + ((k0 / KC) & 1) * PL * CW * LDB;
      if (k0 == 0) __syncthreads();  // s_gcol visible; the previous item's reads done
      for (int idx = tid; idx < CW * kc; idx += NT) {
        const int j = idx / kc, kk = idx - j * kc;
        const long long g = s_gcol[j];
        const long long a = g * XR + k0 + kk;
        sBc[j * LDB + kk] = g >= 0 ? Xin[a] : 0.0;
        if (CPLX) sBc[CW * LDB + j * LDB + kk] = g >= 0 ? Xin[plane + a] : 0.0;
      }
      __syncthreads();
      for (int kb = 0; kb < kc; kb += 4 * kPD) {
#pragma unroll
        for (int d = 0; d < kPD; ++d) {
          const int kk = kb + 4 * d;
          if (kk < kc) {
            double ar[RT], ai[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i) {
              ar[i] = rr[d][i];
              ai[i] = ri[d][i];
            }
            const int kn = k0 + kk + 4 * kPD;
            if (kn < kp) {
#pragma unroll
              for (int i = 0; i < RT; ++i) {
                const int tile = wave + i * NW;
                if (tile < ntiles) {
                  const long long a = (long long)(kn + lq) * ld + tile * 16 + ln;
                  rr[d][i] = Fr[a];
                  if (CPLX) ri[d][i] = Fi[a];
                }
              }
            }
#pragma unroll
            for (int t = 0; t < CT; ++t) {
              const double br = sBc[(t * 16 + ln) * LDB + kk + lq];
              const double bi = CPLX ? sBc[CW * LDB + (t * 16 + ln) * LDB + kk + lq] : 0.0;
#pragma unroll
              for (int i = 0; i < RT; ++i) {
                if (wave + i * NW < ntiles) {
                  acc_r[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br, acc_r[i][t], 0, 0, 0);
                  if (CPLX) {
                    acc_r[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi, acc_r[i][t], 0, 0, 0);
                    acc_i[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi, acc_i[i][t], 0, 0, 0);
                    acc_i[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br, acc_i[i][t], 0, 0, 0);
                  }
                }
              }
            }
          }
        }
      }
    }

    // epilogue: propagator of the next gap, per-column max, rescale, store
    const double* e2 = I.esh + I.eoff[s2];
    double cm[CT];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      cm[t] = 0.0;
      const double dt = s_dt[t * 16 + ln];
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = wave + i * NW;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * q + lq;
            const double p = (m < d_out) ? exp(-dt * e2[m]) : 0.0;
            acc_r[i][t][q] *= p;
            cm[t] = fmax(cm[t], fabs(acc_r[i][t][q]));
            if (CPLX) {
              acc_i[i][t][q] *= p;
              cm[t] = fmax(cm[t], fabs(acc_i[i][t][q]));
            }
          }
        }
      }
      cm[t] = fmax(cm[t], __shfl_xor(cm[t], 16));
      cm[t] = fmax(cm[t], __shfl_xor(cm[t], 32));
      if (lq == 0) s_cmax[wave * CW + t * 16 + ln] = cm[t];
    }
    __syncthreads();
    if (tid < CW) {
      double M = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) M = fmax(M, s_cmax[w2 * CW + tid]);
      int e = 0;
      if (M > 0.0) frexp(M, &e);
      s_e[tid] = e;
      if (s_gcol[tid] >= 0) G.colexp[s_gcol[tid]] += e;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int j = t * 16 + ln;
      const long long g = s_gcol[j];
      if (g < 0) continue;
      const double sc = ldexp(1.0, -s_e[j]);
      double* col = Xout + g * XR;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = wave + i * NW;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * q + lq;
            col[m] = acc_r[i][t][q] * sc;
            if (CPLX) col[plane + m] = acc_i[i][t][q] * sc;
          }
        }
      }
    }
  }
}

// Sectors of any size (beyond the register tile of k_gstep): a work item is
// (group, CW-column tile, RB-row chunk), RB = WR * RT * 16 rows and
// CW = WC * CT * 16 columns; wavefront (wr, wc) of the WR x WC grid computes RT
// row tiles x CT column tiles.  The item's columns of X are staged through LDS
// KC rows at a time, each scaled by its pending power of two as it is loaded
// (exact); F comes from global memory with two k-steps of look-ahead.  The
// epilogue applies the propagator of each column's next gap, stores the
// products unscaled and takes the per-column maximum over the item's rows
// (wavefront, then workgroup reduction), then one device-wide atomicMax per
// column folds it into the round's pending exponent, which the next round
// applies.  The row-chunk-0 item of every column tile also adds the pending
// exponent it consumed to the column's accumulated one and clears the slot
// of the round after next.  Closing strings take the diagonal of F * X from
// the unscaled columns.
template <bool CPLX, int WR, int WC, int RT, int CT, int KC = 32>
__global__ __launch_bounds__(WR * WC * 64) void k_gbig(DevImp I, BatchArgs B, GroupArgs G, int r) {
  constexpr int NW = WR * WC;
  constexpr int NT = NW * 64;
  constexpr int RB = WR * RT * 16;
  constexpr int CW = WC * CT * 16;
  // KC: rows of X staged in LDS per chunk
  constexpr int LDB = KC + 1;            // odd stride: the 16 columns of a B fragment hit distinct banks
  constexpr int PL = CPLX ? 2 : 1;
  __shared__ double sB[2 * PL * CW * LDB];  // two staging buffers: chunk c in buffer c % 2
  __shared__ double s_cmax[WR * CW];
  __shared__ double s_dt[CW];
  __shared__ double s_sc[CW];
  __shared__ long long s_gcol[CW];
  __shared__ int s_item;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int ln = lane & 15, lq = lane >> 4;
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  const int XR = I.xrows;
  const long long T = G.T;
  const long long plane = T * (long long)XR;
  const double* Xin = G.X[(r + 1) & 1];
  double* Xout = G.X[r & 1];
  const int* ep_in = G.epend + (long long)(r % 3) * T;
  int* ep_out = G.epend + (long long)((r + 1) % 3) * T;
  int* ep_clr = G.epend + (long long)((r + 2) % 3) * T;
  const int* istart = G.istart + (long long)r * (NK + 1);
  const int* gstart = G.gstart + (long long)r * (NK + 1);
  const int* hcols = G.hcols + (long long)r * NK;
  const int* colpref = G.colpref + (long long)r * G.S;
  const long long* ritemoff = G.ritemoff;
  typedef double dbl4 __attribute__((ext_vector_type(4)));

  const int n_items = G.n_items[r];
  const int slot = blockIdx.x % kGroupCounters;
  unsigned int* counter = G.counters + ((long long)r * kGroupCounters + slot) * 32;
  for (;;) {
    if (tid == 0) s_item = slot + kGroupCounters * (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= n_items) break;
    const int key = G.item_key[ritemoff[r] + item];
    const bool close = key >= NB;
    const int blk = close ? key - NB : key;
    const int s = blk / I.nops;
    const int s2 = I.next[blk];
    const int d_in = I.dim[s], d_out = I.dim[s2];
    const int ld = (d_out + 15) & ~15;
    const int kp = (d_in + 3) & ~3;
    const double* Fr = I.pool + I.boff[blk];
    const double* Fi = Fr + (long long)ld * kp;

    if (close) {
      // diagonal of F * X: column j of the string meets row j of F; the
      // stored columns are unscaled, their power of two is colexp
      const int cw = G.cw_close;
      const int c0 = (item - istart[key]) * cw;
      const int ncol = min(cw, hcols[key] - c0);
      const long long relbase = G.rcoloff[r] + colpref[gstart[key]] + c0;
      for (int j = wave; j < ncol; j += NW) {
        const long long gcol = G.colg[relbase + j];
        const int jj = (int)G.colaux[relbase + j];
        const double* xr = Xin + gcol * XR;
        double sr = 0.0, si = 0.0;
        for (int k = lane; k < d_in; k += 64) {
          const double fr = Fr[(long long)k * ld + jj], x = xr[k];
          if (CPLX) {
            const double fi = Fi[(long long)k * ld + jj], xi = xr[plane + k];
            sr += fr * x - fi * xi;
            si += fr * xi + fi * x;
          } else {
            sr += fr * x;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        if (lane == 0) {
          PanelRes o;
          o.re = sr;
          o.im = si;
          o.e2 = (double)G.colexp[gcol];
          G.colres[gcol] = o;
        }
      }
      __syncthreads();
      continue;
    }

    const int nrc = (d_out + RB - 1) / RB;
    const int local = item - istart[key];
    const int ct = local / nrc, rc = local - ct * nrc;
    const int c0 = ct * CW;
    const int ncol = min(CW, hcols[key] - c0);
    const long long relbase = G.rcoloff[r] + colpref[gstart[key]] + c0;
    if (tid < CW) {
      const long long g = tid < ncol ? (long long)G.colg[relbase + tid] : -1;
      const int pe = g >= 0 ? ep_in[g] : kNoExp;
      s_gcol[tid] = g;
      s_dt[tid] = tid < ncol ? G.colaux[relbase + tid] : 0.0;
      s_sc[tid] = pe != kNoExp ? ldexp(1.0, -pe) : 1.0;
      if (rc == 0 && g >= 0) {
        if (pe != kNoExp) G.colexp[g] += pe;
        ep_clr[g] = kNoExp;
      }
    }

    dbl4 acc_r[RT][CT], acc_i[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        acc_r[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
        acc_i[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
    const int ntiles = ld >> 4;
    const int tile0 = rc * (RB / 16) + wr * RT;  // first row tile of this wavefront
    // A fragments run kPD k-steps ahead of the products (slot s % kPD)
    constexpr int kPD = 2;
    double rr[kPD][RT], ri[kPD][RT];
#pragma unroll
    for (int d = 0; d < kPD; ++d)
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = tile0 + i;
        rr[d][i] = ri[d][i] = 0.0;
        if (tile < ntiles && 4 * d < kp) {
          const long long a = (long long)(4 * d + lq) * ld + tile * 16 + ln;
          rr[d][i] = Fr[a];
          if (CPLX) ri[d][i] = Fi[a];
        }
      }
    // the next chunk of X is fetched into registers while the current one is multiplied
    constexpr int NPF = (CW * KC + NT - 1) / NT;
    double pf_r[NPF], pf_i[NPF];
    auto fetch = [&](int k0, int kc) {
#pragma unroll
      for (int u = 0; u < NPF; ++u) {
        const int idx = tid + u * NT;
        pf_r[u] = pf_i[u] = 0.0;
        if (idx < CW * kc) {
          const int j = idx / kc, kk = idx - j * kc;
          const long long g = s_gcol[j];
          if (g >= 0) {
            const long long a = g * XR + k0 + kk;
            pf_r[u] = Xin[a] * s_sc[j];
            if (CPLX) pf_i[u] = Xin[plane + a] * s_sc[j];
          }
        }
      }
    };
    __syncthreads();  // column table visible
    fetch(0, min(KC, kp));
    for (int k0 = 0; k0 < kp; k0 += KC) {
      const int kc = min(KC, kp - k0);
      // one barrier per chunk: the buffer written here was last read two chunks
      // ago, and every wavefront finished that chunk before the barrier of the
      // chunk in between
      double* sBc = sB + ((k0 / KC) & 1) * PL * CW * LDB;
#pragma unroll
      for (int u = 0; u < NPF; ++u) {
        const int idx = tid + u * NT;
        if (idx < CW * kc) {
          const int j = idx / kc, kk = idx - j * kc;
          sBc[j * LDB + kk] = pf_r[u];
          if (CPLX) sBc[CW * LDB + j * LDB + kk] = pf_i[u];
        }
      }
      __syncthreads();
      if (k0 + KC < kp) fetch(k0 + KC, min(KC, kp - k0 - KC));
      for (int kb = 0; kb < kc; kb += 4 * kPD) {
#pragma unroll
        for (int d = 0; d < kPD; ++d) {
          const int kk = kb + 4 * d;
          if (kk < kc) {
            double ar[RT], ai[RT];
#pragma unroll
            for (int i = 0; i < RT; ++i) {
              ar[i] = rr[d][i];
              ai[i] = ri[d][i];
            }
            const int kn = k0 + kk + 4 * kPD;
            if (kn < kp) {
#pragma unroll
              for (int i = 0; i < RT; ++i) {
                const int tile = tile0 + i;
                if (tile < ntiles) {
                  const long long a = (long long)(kn + lq) * ld + tile * 16 + ln;
                  rr[d][i] = Fr[a];
                  if (CPLX) ri[d][i] = Fi[a];
                }
              }
            }
#pragma unroll
            for (int t = 0; t < CT; ++t) {
              const int jb = (wc * CT + t) * 16 + ln;
              const double br = sBc[jb * LDB + kk + lq];
              const double bi = CPLX ? sBc[CW * LDB + jb * LDB + kk + lq] : 0.0;
#pragma unroll
              for (int i = 0; i < RT; ++i) {
                if (tile0 + i < ntiles) {
                  acc_r[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br, acc_r[i][t], 0, 0, 0);
                  if (CPLX) {
                    acc_r[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi, acc_r[i][t], 0, 0, 0);
                    acc_i[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi, acc_i[i][t], 0, 0, 0);
                    acc_i[i][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br, acc_i[i][t], 0, 0, 0);
                  }
                }
              }
            }
          }
        }
      }
    }

    // epilogue: propagator of the next gap, per-column max over the item's rows
    const double* e2 = I.esh + I.eoff[s2];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int j = (wc * CT + t) * 16 + ln;
      const double dt = s_dt[j];
      double cm = 0.0;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = tile0 + i;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * q + lq;
            const double p = (m < d_out) ? exp(-dt * e2[m]) : 0.0;
            acc_r[i][t][q] *= p;
            cm = fmax(cm, fabs(acc_r[i][t][q]));
            if (CPLX) {
              acc_i[i][t][q] *= p;
              cm = fmax(cm, fabs(acc_i[i][t][q]));
            }
          }
        }
      }
      cm = fmax(cm, __shfl_xor(cm, 16));
      cm = fmax(cm, __shfl_xor(cm, 32));
      if (lq == 0) s_cmax[wr * CW + j] = cm;
    }
    __syncthreads();
    if (tid < CW && s_gcol[tid] >= 0) {
      double M = 0.0;
      for (int w2 = 0; w2 < WR; ++w2) M = fmax(M, s_cmax[w2 * CW + tid]);
      if (M > 0.0) {
        int e = 0;
        frexp(M, &e);
        atomicMax(ep_out + s_gcol[tid], e);
      }
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int j = (wc * CT + t) * 16 + ln;
      const long long g = s_gcol[j];
      if (g < 0) continue;
      double* col = Xout + g * XR;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = tile0 + i;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * q + lq;
            col[m] = acc_r[i][t][q];
            if (CPLX) col[plane + m] = acc_i[i][t][q];
          }
        }
      }
    }
  }
}

// FP32-split form of k_gbig (same items, staging, pending exponents and
// closes).  Each FP64 product is formed from NSL integer slices of 8 bits per
// operand: F per row, scaled by the row's power of two (rexp) so that |F| < 1;
// X per column, scaled into (-1, 1) by its pending power of two.  With
//   f = sum_s A_s 2^{-8 s},  x = sum_t B_t 2^{-8 t},  |A_s|, |B_t| <= 255,
// the slice products with s + t <= NSL + 1 run on FP32 MFMA 16x16x4 and are
// summed per level L = s + t; a level gets at most NSL (2 NSL complex)
// products below 2^16 per value of k, so over kSplitK values of k its FP32
// sum stays an integer below 2^24 and is exact.  After every such chunk the
// level sums are converted to FP64 and added with weight 2^{-8 L}.  The
// propagators, the rescale and the closes stay FP64.
template <bool CPLX, int NSL>
__host__ __device__ constexpr int split_k() {
  return ((1 << 8) / (NSL * (CPLX ? 2 : 1))) & ~3;
}

template <int NSL>
__device__ __forceinline__ void cut_slices(double v, float* d) {
#pragma unroll
  for (int s = 0; s < NSL; ++s) {
    v *= 256.0;
    const double a = trunc(v);
    d[s] = (float)a;
    v -= a;
  }
}

template <bool CPLX, int WR, int WC, int RT, int CT, int NSL>
__global__ __launch_bounds__(WR * WC * 64) void k_gbig_split(DevImp I, BatchArgs B, GroupArgs G, int r) {
  constexpr int NW = WR * WC;
  constexpr int NT = NW * 64;
  constexpr int RB = WR * RT * 16;
  constexpr int CW = WC * CT * 16;
  constexpr int KC = 32;
  constexpr int LDB = KC + 1;
  constexpr int PL = CPLX ? 2 : 1;
  constexpr int KS = split_k<CPLX, NSL>();  // values of k per exact FP32 chunk (a multiple of 4)
  static_assert(KC % KS == 0 || KS % 4 == 0, "chunking");
  __shared__ double sB[PL * CW * LDB];
  __shared__ double s_cmax[WR * CW];
  __shared__ double s_dt[CW];
  __shared__ double s_sc[CW];
  __shared__ long long s_gcol[CW];
  __shared__ int s_item;
  typedef double dbl4 __attribute__((ext_vector_type(4)));
  typedef float flt4 __attribute__((ext_vector_type(4)));

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WR, wc = wave / WR;
  const int ln = lane & 15, lq = lane >> 4;
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  const int XR = I.xrows;
  const long long T = G.T;
  const long long plane = T * (long long)XR;
  const double* Xin = G.X[(r + 1) & 1];
  double* Xout = G.X[r & 1];
  const int* ep_in = G.epend + (long long)(r % 3) * T;
  int* ep_out = G.epend + (long long)((r + 1) % 3) * T;
  int* ep_clr = G.epend + (long long)((r + 2) % 3) * T;
  const int* istart = G.istart + (long long)r * (NK + 1);
  const int* gstart = G.gstart + (long long)r * (NK + 1);
  const int* hcols = G.hcols + (long long)r * NK;
  const int* colpref = G.colpref + (long long)r * G.S;
  const long long* ritemoff = G.ritemoff;

  const int n_items = G.n_items[r];
  const int slot = blockIdx.x % kGroupCounters;
  unsigned int* counter = G.counters + ((long long)r * kGroupCounters + slot) * 32;
  for (;;) {
    if (tid == 0) s_item = slot + kGroupCounters * (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int item = s_item;
    if (item >= n_items) break;
    const int key = G.item_key[ritemoff[r] + item];
    const bool close = key >= NB;
    const int blk = close ? key - NB : key;
    const int s = blk / I.nops;
    const int s2 = I.next[blk];
    const int d_in = I.dim[s], d_out = I.dim[s2];
    const int ld = (d_out + 15) & ~15;
    const int kp = (d_in + 3) & ~3;
    const double* Fr = I.pool + I.boff[blk];
    const double* Fi = Fr + (long long)ld * kp;

    if (close) {
      const int cw = G.cw_close;
      const int c0 = (item - istart[key]) * cw;
      const int ncol = min(cw, hcols[key] - c0);
      const long long relbase = G.rcoloff[r] + colpref[gstart[key]] + c0;
      for (int j = wave; j < ncol; j += NW) {
        const long long gcol = G.colg[relbase + j];
        const int jj = (int)G.colaux[relbase + j];
        const double* xr = Xin + gcol * XR;
        double sr = 0.0, si = 0.0;
        for (int k = lane; k < d_in; k += 64) {
          const double fr = Fr[(long long)k * ld + jj], x = xr[k];
          if (CPLX) {
            const double fi = Fi[(long long)k * ld + jj], xi = xr[plane + k];
            sr += fr * x - fi * xi;
            si += fr * xi + fi * x;
          } else {
            sr += fr * x;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        if (lane == 0) {
          PanelRes o;
          o.re = sr;
          o.im = si;
          o.e2 = (double)G.colexp[gcol];
          G.colres[gcol] = o;
        }
      }
      __syncthreads();
      continue;
    }

    const int nrc = (d_out + RB - 1) / RB;
    const int local = item - istart[key];
    const int ct = local / nrc, rc = local - ct * nrc;
    const int c0 = ct * CW;
    const int ncol = min(CW, hcols[key] - c0);
    const long long relbase = G.rcoloff[r] + colpref[gstart[key]] + c0;
    if (tid < CW) {
      const long long g = tid < ncol ? (long long)G.colg[relbase + tid] : -1;
      const int pe = g >= 0 ? ep_in[g] : kNoExp;
      s_gcol[tid] = g;
      s_dt[tid] = tid < ncol ? G.colaux[relbase + tid] : 0.0;
      s_sc[tid] = pe != kNoExp ? ldexp(1.0, -pe) : 1.0;
      if (rc == 0 && g >= 0) {
        if (pe != kNoExp) G.colexp[g] += pe;
        ep_clr[g] = kNoExp;
      }
    }
    const short* rex = I.rexp + I.roff[blk];
    const int ntiles = ld >> 4;
    const int tile0 = rc * (RB / 16) + wr * RT;
    // inverse row scales of the A rows this lane feeds (row tile*16 + ln)
    double ainv[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) ainv[i] = (tile0 + i < ntiles) ? ldexp(1.0, -(int)rex[(tile0 + i) * 16 + ln]) : 0.0;

    dbl4 acc_r[RT][CT], acc_i[RT][CT];
    flt4 lr[RT][CT][NSL], li[RT][CT][NSL];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int t = 0; t < CT; ++t) {
        acc_r[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
        acc_i[i][t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int L = 0; L < NSL; ++L) {
          lr[i][t][L] = flt4{0.f, 0.f, 0.f, 0.f};
          li[i][t][L] = flt4{0.f, 0.f, 0.f, 0.f};
        }
      }
    int in_chunk = 0;  // values of k summed into the FP32 levels since the last flush
    for (int k0 = 0; k0 < kp; k0 += KC) {
      const int kc = min(KC, kp - k0);
      __syncthreads();
      for (int idx = tid; idx < CW * kc; idx += NT) {
        const int j = idx / kc, kk = idx - j * kc;
        const long long g = s_gcol[j];
        const long long a = g * XR + k0 + kk;
        sB[j * LDB + kk] = g >= 0 ? Xin[a] * s_sc[j] : 0.0;
        if (CPLX) sB[CW * LDB + j * LDB + kk] = g >= 0 ? Xin[plane + a] * s_sc[j] : 0.0;
      }
      __syncthreads();
      for (int kk = 0; kk < kc; kk += 4) {
        float afr[RT][NSL], afi[RT][NSL];
#pragma unroll
        for (int i = 0; i < RT; ++i) {
          const int tile = tile0 + i;
          double vr = 0.0, vi = 0.0;
          if (tile < ntiles) {
            const long long a = (long long)(k0 + kk + lq) * ld + tile * 16 + ln;
            vr = Fr[a] * ainv[i];
            if (CPLX) vi = Fi[a] * ainv[i];
          }
          cut_slices<NSL>(vr, afr[i]);
          if (CPLX) cut_slices<NSL>(vi, afi[i]);
        }
#pragma unroll
        for (int t = 0; t < CT; ++t) {
          const int jb = (wc * CT + t) * 16 + ln;
          float bxr[NSL], bxi[NSL];
          cut_slices<NSL>(sB[jb * LDB + kk + lq], bxr);
          if (CPLX) cut_slices<NSL>(sB[CW * LDB + jb * LDB + kk + lq], bxi);
#pragma unroll
          for (int i = 0; i < RT; ++i) {
            if (tile0 + i < ntiles) {
              // level L = s + t (slice indices from 1), kept for L <= NSL + 1
#pragma unroll
              for (int L = 2; L <= NSL + 1; ++L) {
#pragma unroll
                for (int s1 = 1; s1 < L; ++s1) {
                  const int t1 = L - s1;
                  lr[i][t][L - 2] =
                      __builtin_amdgcn_mfma_f32_16x16x4f32(afr[i][s1 - 1], bxr[t1 - 1], lr[i][t][L - 2], 0, 0, 0);
                  if (CPLX) {
                    lr[i][t][L - 2] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(-afi[i][s1 - 1], bxi[t1 - 1], lr[i][t][L - 2], 0, 0, 0);
                    li[i][t][L - 2] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(afr[i][s1 - 1], bxi[t1 - 1], li[i][t][L - 2], 0, 0, 0);
                    li[i][t][L - 2] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(afi[i][s1 - 1], bxr[t1 - 1], li[i][t][L - 2], 0, 0, 0);
                  }
                }
              }
            }
          }
        }
        in_chunk += 4;
        if (in_chunk == KS || k0 + kk + 4 >= kp) {
          // exact FP32 level sums -> FP64 with weights 2^{-8 L}
#pragma unroll
          for (int i = 0; i < RT; ++i)
#pragma unroll
            for (int t = 0; t < CT; ++t)
#pragma unroll
              for (int L = 2; L <= NSL + 1; ++L) {
                const double wgt = ldexp(1.0, -8 * L);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                  acc_r[i][t][q] += (double)lr[i][t][L - 2][q] * wgt;
                  if (CPLX) acc_i[i][t][q] += (double)li[i][t][L - 2][q] * wgt;
                }
                lr[i][t][L - 2] = flt4{0.f, 0.f, 0.f, 0.f};
                li[i][t][L - 2] = flt4{0.f, 0.f, 0.f, 0.f};
              }
          in_chunk = 0;
        }
      }
    }

    // epilogue: row scales back, propagator of the next gap, per-column max;
    // item q of lane l in the FP32 result is row 4 (l / 16) + q, column l % 16
    const double* e2 = I.esh + I.eoff[s2];
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int j = (wc * CT + t) * 16 + ln;
      const double dt = s_dt[j];
      double cm = 0.0;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = tile0 + i;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * lq + q;
            const double p = (m < d_out) ? ldexp(exp(-dt * e2[m]), (int)rex[m]) : 0.0;
            acc_r[i][t][q] *= p;
            cm = fmax(cm, fabs(acc_r[i][t][q]));
            if (CPLX) {
              acc_i[i][t][q] *= p;
              cm = fmax(cm, fabs(acc_i[i][t][q]));
            }
          }
        }
      }
      cm = fmax(cm, __shfl_xor(cm, 16));
      cm = fmax(cm, __shfl_xor(cm, 32));
      if (lq == 0) s_cmax[wr * CW + j] = cm;
    }
    __syncthreads();
    if (tid < CW && s_gcol[tid] >= 0) {
      double M = 0.0;
      for (int w2 = 0; w2 < WR; ++w2) M = fmax(M, s_cmax[w2 * CW + tid]);
      if (M > 0.0) {
        int e = 0;
        frexp(M, &e);
        atomicMax(ep_out + s_gcol[tid], e);
      }
    }
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      const int j = (wc * CT + t) * 16 + ln;
      const long long g = s_gcol[j];
      if (g < 0) continue;
      double* col = Xout + g * XR;
#pragma unroll
      for (int i = 0; i < RT; ++i) {
        const int tile = tile0 + i;
        if (tile < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = tile * 16 + 4 * lq + q;
            col[m] = acc_r[i][t][q];
            if (CPLX) col[plane + m] = acc_i[i][t][q];
          }
        }
      }
    }
  }
}

// Sectors of at most 16 * MT states: one wavefront per work item of 16 * CT
// columns of one group, all row tiles in registers, no workgroup barrier.
// Lane l supplies A[row l%16][k l/16] and B[k l/16][column l%16]; item q of
// the 16x16x4 result is row 4q + l/16, column l%16, so the per-column max is
// a reduction over the four lanes of a column (xor 16, 32).
template <bool CPLX, int MT, int CT>
__global__ __launch_bounds__(256, CT == 1 ? 3 : 2) void k_gstep_wave(DevImp I, BatchArgs B, GroupArgs G, int r) {
  const int lane = threadIdx.x & 63;
  const int ln = lane & 15, lq = lane >> 4;
  const int NB = I.n_sec * I.nops, NK = 2 * NB;
  const int XR = I.xrows;
  const long long plane = G.T * (long long)XR;
  const double* Xin = G.X[(r + 1) & 1];
  double* Xout = G.X[r & 1];
  const int* istart = G.istart + (long long)r * (NK + 1);
  const int* gstart = G.gstart + (long long)r * (NK + 1);
  const int* hcols = G.hcols + (long long)r * NK;
  const int* colpref = G.colpref + (long long)r * G.S;
  const int* item_key = G.item_key + G.ritemoff[r];
  const long long rcoloff = G.rcoloff[r];
  typedef double dbl4 __attribute__((ext_vector_type(4)));
  // propagators of the item's distinct gaps (the columns of one string share
  // its gap): kRuns runs of equal gaps x 16 * MT rows per wavefront, one
  // 16-column tile at a time
  constexpr int kRuns = 8;
  __shared__ double s_prop[4][kRuns * 16 * MT];
  __shared__ double s_gap[4][kRuns];
  const int wv = threadIdx.x >> 6;

  // item i is served by counter i % kGroupCounters
  const int n_items = G.n_items[r];
  const int slot = (blockIdx.x * 4 + (threadIdx.x >> 6)) % kGroupCounters;
  unsigned int* counter = G.counters + ((long long)r * kGroupCounters + slot) * 32;
  for (;;) {
    int item = 0;
    if (lane == 0) item = slot + kGroupCounters * (int)atomicAdd(counter, 1u);
    item = __shfl(item, 0);
    if (item >= n_items) break;
    const int key = item_key[item];
    const bool close = key >= NB;
    const int blk = close ? key - NB : key;
    const int cw = close ? G.cw_close : 16 * CT;
    const int c0 = (item - istart[key]) * cw;
    const int ncol = min(cw, hcols[key] - c0);
    const long long relbase = rcoloff + colpref[gstart[key]] + c0;
    const int s = blk / I.nops;
    const int s2 = I.next[blk];
    const int d_in = I.dim[s], d_out = I.dim[s2];
    const int ld = (d_out + 15) & ~15;
    const int kp = (d_in + 3) & ~3;
    const double* Fr = I.pool + I.boff[blk];
    const double* Fi = Fr + (long long)ld * kp;

    if (close) {
      for (int j = 0; j < ncol; ++j) {
        const long long gc = G.colg[relbase + j];
        const int jj = (int)G.colaux[relbase + j];
        const double* xc = Xin + gc * XR;
        double sr = 0.0, si = 0.0;
        for (int k = lane; k < d_in; k += 64) {
          const double fr = Fr[(long long)k * ld + jj], x = xc[k];
          if (CPLX) {
            const double fi = Fi[(long long)k * ld + jj], xi = xc[plane + k];
            sr += fr * x - fi * xi;
            si += fr * xi + fi * x;
          } else {
            sr += fr * x;
          }
        }
        for (int off = 32; off > 0; off >>= 1) {
          sr += __shfl_xor(sr, off);
          si += __shfl_xor(si, off);
        }
        if (lane == 0) {
          PanelRes o;
          o.re = sr;
          o.im = si;
          o.e2 = (double)G.colexp[gc];
          G.colres[gc] = o;
        }
      }
      continue;
    }

    // column tile c holds the item's columns 16 c .. 16 c + 15, lane column ln
    bool live[CT];
    long long gcol[CT];
    double dt[CT];
    const double* xr[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      live[c] = ln + 16 * c < ncol;
      gcol[c] = live[c] ? (long long)G.colg[relbase + 16 * c + ln] : 0;
      dt[c] = live[c] ? G.colaux[relbase + 16 * c + ln] : 0.0;
      xr[c] = Xin + gcol[c] * XR;
    }
    const int ntiles = ld >> 4;
    dbl4 acc_r[CT][MT], acc_i[CT][MT];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        acc_r[c][t] = dbl4{0.0, 0.0, 0.0, 0.0};
        acc_i[c][t] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
    // operands of the next k-step are loaded while the current one multiplies;
    // one A fragment serves every column tile
    double nar[MT], nai[MT], nbr[CT], nbi[CT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      nar[t] = nai[t] = 0.0;
      if (t < ntiles) {
        nar[t] = Fr[(long long)lq * ld + t * 16 + ln];
        if (CPLX) nai[t] = Fi[(long long)lq * ld + t * 16 + ln];
      }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      nbr[c] = live[c] ? xr[c][lq] : 0.0;
      nbi[c] = (CPLX && live[c]) ? xr[c][plane + lq] : 0.0;
    }
    for (int k0 = 0; k0 < kp; k0 += 4) {
      double ar[MT], ai[MT], br[CT], bi[CT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        ar[t] = nar[t];
        ai[t] = nai[t];
      }
#pragma unroll
      for (int c = 0; c < CT; ++c) {
        br[c] = nbr[c];
        bi[c] = nbi[c];
      }
      const int kn = k0 + 4;
      if (kn < kp) {
        const long long row = (long long)(kn + lq) * ld;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t < ntiles) {
            nar[t] = Fr[row + t * 16 + ln];
            if (CPLX) nai[t] = Fi[row + t * 16 + ln];
          }
        }
#pragma unroll
        for (int c = 0; c < CT; ++c) {
          nbr[c] = live[c] ? xr[c][kn + lq] : 0.0;
          nbi[c] = (CPLX && live[c]) ? xr[c][plane + kn + lq] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (t < ntiles) {
#pragma unroll
          for (int c = 0; c < CT; ++c) {
            acc_r[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[t], br[c], acc_r[c][t], 0, 0, 0);
            if (CPLX) {
              acc_r[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[t], bi[c], acc_r[c][t], 0, 0, 0);
              acc_i[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[t], bi[c], acc_i[c][t], 0, 0, 0);
              acc_i[c][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[t], br[c], acc_i[c][t], 0, 0, 0);
            }
          }
        }
      }
    }

    // per column tile: propagator of the next gap, per-column max, rescale, store
    const double* e2 = I.esh + I.eoff[s2];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      // runs of equal gaps among the tile's columns (ballot over the lanes of row quarter 0)
      const double dt_left = __shfl(dt[c], (lane + 63) & 63);
      const unsigned long long starts =
          __ballot(lq == 0 && live[c] && (ln == 0 || dt[c] != dt_left)) & 0xffffull;
      const int n_runs = __popcll(starts);
      const int run = __popcll(starts & ((2ull << ln) - 1)) - 1;
      const bool tab = n_runs <= kRuns;
      if (tab) {
        // every lane is done reading the previous tile's table before it is rewritten
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lq == 0 && ((starts >> ln) & 1)) s_gap[wv][run] = dt[c];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int u = 0; u < n_runs; ++u) {
          const double g = s_gap[wv][u];
          for (int m = lane; m < ld; m += 64) s_prop[wv][u * 16 * MT + m] = (m < d_out) ? exp(-g * e2[m]) : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      const double* prop = &s_prop[wv][(run > 0 ? run : 0) * 16 * MT];
      double cm = 0.0;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (t < ntiles) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int m = t * 16 + 4 * q + lq;
            const double p = tab ? prop[m] : ((m < d_out) ? exp(-dt[c] * e2[m]) : 0.0);
            acc_r[c][t][q] *= p;
            cm = fmax(cm, fabs(acc_r[c][t][q]));
            if (CPLX) {
              acc_i[c][t][q] *= p;
              cm = fmax(cm, fabs(acc_i[c][t][q]));
            }
          }
        }
      }
      cm = fmax(cm, __shfl_xor(cm, 16));
      cm = fmax(cm, __shfl_xor(cm, 32));
      int e = 0;
      if (cm > 0.0) frexp(cm, &e);
      const double sc = ldexp(1.0, -e);
      if (live[c]) {
        if (lq == 0) G.colexp[gcol[c]] += e;
        double* col = Xout + gcol[c] * XR;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t < ntiles) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int m = t * 16 + 4 * q + lq;
              col[m] = acc_r[c][t][q] * sc;
              if (CPLX) col[plane + m] = acc_i[c][t][q] * sc;
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// combine
// ---------------------------------------------------------------------------
// One wavefront per configuration: lanes over the columns of each string.
__global__ __launch_bounds__(256) void k_gcombine(DevImp I, BatchArgs B, GroupArgs G) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= B.n_cfg) return;
  ctr_value v;
  v.re = v.im = v.log_scale = 0.0;
  v.log_abs = -INFINITY;
  const int flags = B.cfg_flags[c];
  v.flags = flags;
  v.n_strings = B.cfg_nstr[c];
  v.log_bound = B.cfg_logB[c];
  if (!(flags & (CTR_FLAG_INVALID | CTR_FLAG_REJECTED | CTR_FLAG_ZERO))) {
    const double ln2 = 0.69314718055994530942;
    const StrRec* recs = B.rec + (long long)c * I.n_sec;
    double lmax = -INFINITY;
    for (int q = 0; q < I.n_sec; ++q) {
      const StrRec R = recs[q];
      if (R.n_panels == 0) continue;
      const long long cb = G.s_colbase[B.cfg_off[c] + R.loc_off];
      for (int j = lane; j < R.width; j += 64) {
        const PanelRes P = G.colres[cb + j];
        if (P.re != 0.0 || P.im != 0.0) lmax = fmax(lmax, P.e2 * ln2 - R.L);
      }
    }
    for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off));
    if (lmax > -INFINITY) {
      double sr = 0.0, si = 0.0, sa = 0.0;
      for (int q = 0; q < I.n_sec; ++q) {
        const StrRec R = recs[q];
        if (R.n_panels == 0) continue;
        const long long cb = G.s_colbase[B.cfg_off[c] + R.loc_off];
        for (int j = lane; j < R.width; j += 64) {
          const PanelRes P = G.colres[cb + j];
          if (P.re != 0.0 || P.im != 0.0) {
            const double f = exp(P.e2 * ln2 - R.L - lmax);
            sr += P.re * f;
            si += P.im * f;
            sa += hypot(P.re, P.im) * f;
          }
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
        sa += __shfl_xor(sa, off);
      }
      v.re = sr;
      v.im = si;
      v.log_scale = lmax - I.beta * I.E0;
      v.log_abs = log(sa) + v.log_scale;
    }
  }
  if (lane == 0) B.out[c] = v;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

struct GVariant {
  const void* fn;
  int nw, cw;
  int rchunk;  // rows per product item (0: all rows)
};

template <bool CPLX, int NW, int RT, int CT>
GVariant make_gvariant() {
  return GVariant{reinterpret_cast<const void*>(&k_gstep<CPLX, NW, RT, CT>), NW, CT * 16, 0};
}

template <bool CPLX, int MT, int CT = 1>
GVariant make_wvariant() {
  return GVariant{reinterpret_cast<const void*>(&k_gstep_wave<CPLX, MT, CT>), 4, 16 * CT, 0};
}

template <bool CPLX, int WR, int WC, int RT, int CT, int KC = 32>
GVariant make_bvariant() {
  return GVariant{reinterpret_cast<const void*>(&k_gbig<CPLX, WR, WC, RT, CT, KC>), WR * WC, WC * CT * 16,
                  WR * RT * 16};
}

// FP32-split items: 8 wavefronts x one row tile x one column tile (128 rows x 16 columns); on the
// crystal-field f-shell (16 configurations, 7 slices) 1.08 traces/s against 1.04 for 8 x 1 x 2 and 0.91 for
// 4 x 2 wavefronts of 1 x 2 tiles (the level accumulators leave room for few tiles per wavefront)
template <bool CPLX, int NSL>
GVariant make_svariant() {
  constexpr int WR = 8, WC = 1, RT = 1, CT = 1;
  return GVariant{reinterpret_cast<const void*>(&k_gbig_split<CPLX, WR, WC, RT, CT, NSL>), WR * WC, WC * CT * 16,
                  WR * RT * 16};
}

// Small sectors: one wavefront per item of 16 or 32 columns (all row tiles
// in registers); up to 384 rows: a workgroup per 32/64-column item, rows split
// over its wavefronts; larger: row-chunked items (k_gbig).  alt = 1 selects
// the other measured tile shape where there is one (the autotuner times
// both); false if there is none.  alt = 2, 3: the row-chunked shapes at any
// size.
bool pick_gvariant(const DevImp& imp, int alt, GVariant* v, int split = 0) {
  const int tiles = imp.xrows / 16;
  if (split) {
    // FP32-split products: row-chunked items only (6 or 7 slices)
    if (split != 6 && split != 7) return false;
    if (imp.is_complex) *v = split == 7 ? make_svariant<true, 7>() : make_svariant<true, 6>();
    else *v = split == 7 ? make_svariant<false, 7>() : make_svariant<false, 6>();
    return alt == 2;
  }
  if (alt >= 2) {
    // row-chunked items at any size (alt 2 and 3: the two tile shapes).  A sweep of 14 shapes on the
    // crystal-field f-shell (200 configurations) put 16 wavefronts x one row tile x two column tiles
    // (256 rows x 32 columns, 4 wavefronts per SIMD) first at 16.0 traces/s, 8 x 2 x 2 at 14.4,
    // 4 x 2 column groups of 2 x 2 at 12.3; with the staging double-buffered, chunks of 16 rows of X
    // reach 16.4 (32 rows: 16.0, 8 rows spill)
    if (imp.is_complex) *v = alt == 3 ? make_bvariant<true, 8, 1, 2, 2>() : make_bvariant<true, 16, 1, 1, 2, 16>();
    else *v = alt == 3 ? make_bvariant<false, 8, 1, 2, 2>() : make_bvariant<false, 16, 1, 1, 2>();
    return alt <= 3;
  }
  if (imp.is_complex) {
    if (tiles <= 2) *v = make_wvariant<true, 2>();
    else if (tiles <= 8) *v = make_gvariant<true, 4, 2, 2>();
    else if (tiles <= 24) *v = alt ? make_gvariant<true, 8, 3, 2>() : make_gvariant<true, 12, 2, 2>();
    else *v = alt ? make_bvariant<true, 8, 1, 2, 2>() : make_bvariant<true, 16, 1, 1, 2, 16>();
    return !alt || tiles > 8;
  }
  if (tiles <= 2) *v = make_wvariant<false, 2>();
  else if (tiles <= 4) *v = make_wvariant<false, 4>();
  else if (tiles <= 8) *v = alt ? make_wvariant<false, 8, 1>() : make_wvariant<false, 8, 2>();
  else if (tiles <= 24) *v = make_gvariant<false, 8, 3, 4>();
  else *v = alt ? make_bvariant<false, 8, 1, 2, 2>() : make_bvariant<false, 16, 1, 1, 2>();
  return !alt || (tiles > 4 && tiles <= 8) || tiles > 24;
}

}  // namespace

int group_grid(const DevImp& imp, int device, int alt, int* cw_step, int* rchunk_out, int split) {
  GVariant v;
  if (!pick_gvariant(imp, alt, &v, split)) return 0;
  if (rchunk_out) *rchunk_out = v.rchunk;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, v.fn, v.nw * 64, 0) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) return 0;
  if (cw_step) *cw_step = v.cw;
  const int grid = per_cu > 0 ? per_cu * cus : 0;
  return grid >= kGroupCounters ? grid : 0;  // every counter needs at least one worker
}

hipError_t launch_group_prepare(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, long long max_strings,
                                hipStream_t stream) {
  if (max_strings > 0)
    hipLaunchKernelGGL(k_gstrings, dim3((unsigned)((max_strings + 255) / 256)), dim3(256), 0, stream, imp, b, g);
  hipLaunchKernelGGL(k_gscan1, dim3(1), dim3(1024), 0, stream, imp, b, g);
  return hipGetLastError();
}

hipError_t launch_group_schedule(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, hipStream_t stream) {
  const unsigned sb = (unsigned)((g.S + 255) / 256);
  if (g.S > 0) hipLaunchKernelGGL(k_gwalk, dim3(sb), dim3(256), 0, stream, imp, b, g, 0);
  if (g.R > 1) hipLaunchKernelGGL(k_gsched, dim3(g.R - 1), dim3(1024), 0, stream, imp, g);
  if (g.S > 0) hipLaunchKernelGGL(k_gwalk, dim3(sb), dim3(256), 0, stream, imp, b, g, 1);
  if (g.R > 1) {
    hipLaunchKernelGGL(k_gcolpref, dim3(g.R - 1), dim3(1024), 0, stream, imp, b, g);
    hipLaunchKernelGGL(k_gscan2, dim3(1), dim3(1024), 0, stream, g);
    const long long nk = (long long)(g.R - 1) * 2 * imp.n_sec * imp.nops;
    hipLaunchKernelGGL(k_gkeys, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, stream, imp, g);
    const long long ns = (long long)(g.R - 1) * g.S;
    if (ns > 0) hipLaunchKernelGGL(k_gitems, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, stream, imp, b, g);
  }
  if (g.S > 0) {
    if (g.rchunk > 0) {
      if (imp.is_complex)
        hipLaunchKernelGGL(k_gfirst_big<true>, dim3((unsigned)g.S), dim3(256), 0, stream, imp, b, g);
      else
        hipLaunchKernelGGL(k_gfirst_big<false>, dim3((unsigned)g.S), dim3(256), 0, stream, imp, b, g);
    } else if (imp.is_complex) {
      hipLaunchKernelGGL(k_gfirst<true>, dim3((unsigned)g.S), dim3(256), 0, stream, imp, b, g);
    } else {
      hipLaunchKernelGGL(k_gfirst<false>, dim3((unsigned)g.S), dim3(256), 0, stream, imp, b, g);
    }
  }
  return hipGetLastError();
}

hipError_t launch_group_round(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, int r, int grid, int alt,
                              int split, hipStream_t stream) {
  GVariant v;
  if (!pick_gvariant(imp, alt, &v, split) || grid <= 0) return hipErrorInvalidValue;
  if (v.cw != g.cw_step || v.rchunk != g.rchunk) return hipErrorInvalidValue;  // schedule built for another shape
  void* args[] = {const_cast<DevImp*>(&imp), const_cast<BatchArgs*>(&b), const_cast<GroupArgs*>(&g), &r};
  return hipLaunchKernel(v.fn, dim3(grid), dim3(v.nw * 64), args, 0, stream);
}

hipError_t group_round_node(const DevImp& imp, const GroupArgs& g, int grid, int alt, int split, void** args,
                            hipKernelNodeParams* p) {
  GVariant v;
  if (!pick_gvariant(imp, alt, &v, split) || grid <= 0) return hipErrorInvalidValue;
  if (v.cw != g.cw_step || v.rchunk != g.rchunk) return hipErrorInvalidValue;
  p->func = const_cast<void*>(v.fn);
  p->gridDim = dim3(grid);
  p->blockDim = dim3(v.nw * 64);
  p->sharedMemBytes = 0;
  p->kernelParams = args;
  p->extra = nullptr;
  return hipSuccess;
}

hipError_t launch_group_combine(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, hipStream_t stream) {
  if (b.n_cfg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gcombine, dim3((b.n_cfg + 3) / 4), dim3(256), 0, stream, imp, b, g);
  return hipGetLastError();
}

}  // namespace ctr
