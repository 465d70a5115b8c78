// Markov chains around the local trace (ctr_mc_* in include/ctrace.h).
//
// Sec. 2.3.1 (sampling), App. C (Metropolis-Hastings with the uniform drawn
// first), App. D (Pauli-aware pair insertion and removal), Sec. 2.2 (w_hyb as
// a determinant of the hybridisation function).  The hybridisation part runs
// on the host with fast updates of each flavor's inverse matrix (O(k^2) per
// move); the local traces of all chains' proposals go to the device as one
// lazy batch per step, whose threshold carries the rest of the acceptance
// ratio, so proposals that cannot be accepted stop at their bound.
//
// Proposal weights (reading of App. D, from detailed balance for two uniform
// times inside the chosen interval): insertion into an interval of length d
// after one of the N operators of the flavor, q = N d^2 / (2 (N + 2)); into
// an empty flavor, q = beta^2; removal, the inverses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ctrace_internal.h"

namespace {

// One flavor's hybridisation block: M[r][s] = Delta(tc[r] - ta[s]) over its
// creators (rows) and annihilators (columns), in insertion order, and its
// inverse inv[s * k + r] = (M^-1)[s][r].
struct FlavorDet {
  std::vector<double> tc, ta, inv;
  int k = 0;
  int updates = 0;
  double ld = 0.0;  // log |det M|
};

struct Chain {
  std::vector<double> tau;
  std::vector<int32_t> op;
  std::vector<FlavorDet> fl;
  double la_loc = 0.0;  // log |w_loc|
  double la_hyb = 0.0;  // log |w_hyb|
};

// A pending move of one chain.
struct Move {
  int kind = -1;  // -1 none, 0 insert, 1 remove
  int f = 0;
  double q = 0.0, ratio = 0.0;
  double tc = 0.0, ta = 0.0;  // insert: new creator / annihilator times
  int ic = -1, ia = -1;       // remove: positions in tau/op of the creator / annihilator
  int rc = -1, ra = -1;       // remove: row (creator) and column (annihilator) in the flavor block
  std::vector<double> v, w;   // insert: inv * Q and R * inv
};

// Persistent workers for the per-chain host passes: run(n, f) calls f(i) for
// i in [0, n) on all workers and the caller, in chunks taken from a shared
// counter, and returns when every index is done.
class Pool {
 public:
  explicit Pool(int workers) {
    for (int w = 0; w < workers; ++w) threads_.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : threads_) t.join();
  }
  void run(int n, const std::function<void(int)>& f) {
    if (threads_.empty() || n < 64) {
      for (int i = 0; i < n; ++i) f(i);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(m_);
      f_ = &f;
      n_ = n;
      next_.store(0);
      busy_ = (int)threads_.size();
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(m_);
    done_cv_.wait(lk, [this] { return busy_ == 0; });
    f_ = nullptr;
  }

 private:
  static constexpr int kChunk = 32;
  void work() {
    for (;;) {
      const int i0 = next_.fetch_add(kChunk);
      if (i0 >= n_) return;
      const int i1 = std::min(n_, i0 + kChunk);
      for (int i = i0; i < i1; ++i) (*f_)(i);
    }
  }
  void loop() {
    long long seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
      {
        std::lock_guard<std::mutex> lk(m_);
        --busy_;
      }
      done_cv_.notify_one();
    }
  }
  std::vector<std::thread> threads_;
  std::mutex m_;
  std::condition_variable cv_, done_cv_;
  const std::function<void(int)>* f_ = nullptr;
  int n_ = 0, busy_ = 0;
  long long gen_ = 0;
  bool stop_ = false;
  std::atomic<int> next_{0};
};

}  // namespace

struct ctr_mc {
  ctr_ctx* ctx = nullptr;
  int nf = 0, nb = 0;
  double beta = 0.0;
  int rebuild_every = 64;
  bool full = false;  // full trace batches instead of lazy ones
  std::vector<double> eps, vv;  // [nf * nb]
  std::vector<Chain> chains;
  std::vector<Move> moves;
  long long n_steps = 0, n_proposed = 0, n_lazy_rejected = 0, n_accepted = 0;
  double host_ms = 0.0, trace_ms = 0.0;  // wall time of the host passes and of the trace batches
  // batch buffers
  std::vector<int64_t> offs;
  std::vector<double> btau, thr;
  std::vector<int32_t> bop, bchain;
  std::vector<ctr_value> out;
  std::vector<double> thr_c;       // per chain: threshold of its proposal
  std::vector<int64_t> len_c;      // per chain: operators of its proposal, -1 if it is not evaluated
  std::vector<int32_t> slot_c;     // per chain: its index in the batch, -1 if none
  std::vector<int32_t> acc_c;      // per chain: 1 if the move was accepted this step
  std::unique_ptr<Pool> pool;
};

namespace {

// Delta_f(x) for x in (-beta, beta), x != 0: -sum_k V^2 e^{-x eps}/(1 + e^{-beta eps})
// on (0, beta), antiperiodic below; written so that no exponent is positive.
double delta(const ctr_mc* mc, int f, double x) {
  double sign = 1.0;
  if (x < 0.0) {
    x += mc->beta;
    sign = -1.0;
  }
  double total = 0.0;
  for (int k = 0; k < mc->nb; ++k) {
    const double e = mc->eps[f * mc->nb + k], a = mc->vv[f * mc->nb + k];
    const double term = e >= 0.0 ? std::exp(-x * e) / (1.0 + std::exp(-mc->beta * e))
                                 : std::exp((mc->beta - x) * e) / (std::exp(mc->beta * e) + 1.0);
    total += a * a * term;
  }
  return -sign * total;
}

// Inverse and log|det| of the flavor block from scratch (Gauss-Jordan,
// partial pivoting).  Returns false if the block is singular.
bool rebuild(const ctr_mc* mc, int f, FlavorDet& D, double* log_det) {
  const int k = D.k;
  std::vector<double> a((size_t)k * k), b((size_t)k * k, 0.0);
  for (int r = 0; r < k; ++r)
    for (int s = 0; s < k; ++s) a[(size_t)r * k + s] = delta(mc, f, D.tc[r] - D.ta[s]);
  for (int i = 0; i < k; ++i) b[(size_t)i * k + i] = 1.0;
  double ld = 0.0;
  for (int c = 0; c < k; ++c) {
    int p = c;
    for (int r = c + 1; r < k; ++r)
      if (std::fabs(a[(size_t)r * k + c]) > std::fabs(a[(size_t)p * k + c])) p = r;
    const double piv = a[(size_t)p * k + c];
    if (piv == 0.0) return false;
    if (p != c)
      for (int j = 0; j < k; ++j) {
        std::swap(a[(size_t)p * k + j], a[(size_t)c * k + j]);
        std::swap(b[(size_t)p * k + j], b[(size_t)c * k + j]);
      }
    ld += std::log(std::fabs(piv));
    const double ip = 1.0 / piv;
    for (int j = 0; j < k; ++j) {
      a[(size_t)c * k + j] *= ip;
      b[(size_t)c * k + j] *= ip;
    }
    for (int r = 0; r < k; ++r) {
      if (r == c) continue;
      const double m = a[(size_t)r * k + c];
      if (m == 0.0) continue;
      for (int j = 0; j < k; ++j) {
        a[(size_t)r * k + j] -= m * a[(size_t)c * k + j];
        b[(size_t)r * k + j] -= m * b[(size_t)c * k + j];
      }
    }
  }
  // b = M^-1 with rows indexed like M's columns: b[s][r]
  D.inv.swap(b);
  D.updates = 0;
  *log_det = ld;
  return true;
}

// Builds the flavor blocks and w_hyb of a chain from its operator list.
bool build_hyb(const ctr_mc* mc, Chain& C) {
  C.fl.assign(mc->nf, FlavorDet{});
  for (size_t i = 0; i < C.op.size(); ++i) {
    FlavorDet& D = C.fl[C.op[i] >> 1];
    (C.op[i] & 1 ? D.tc : D.ta).push_back(C.tau[i]);
  }
  C.la_hyb = 0.0;
  for (int f = 0; f < mc->nf; ++f) {
    FlavorDet& D = C.fl[f];
    if (D.tc.size() != D.ta.size()) return false;
    D.k = (int)D.tc.size();
    D.ld = 0.0;
    if (D.k > 0 && !rebuild(mc, f, D, &D.ld)) return false;
    C.la_hyb += D.ld;
  }
  return true;
}

bool time_taken(const Chain& C, double t) { return std::binary_search(C.tau.begin(), C.tau.end(), t); }

// The move drawn by u[0..5] (same draws as the method's description above).
void propose(const ctr_mc* mc, const Chain& C, const double* u, Move& m) {
  m.kind = -1;
  const int f = std::min(mc->nf - 1, (int)(u[1] * mc->nf));
  m.f = f;
  std::vector<int> L;
  for (size_t i = 0; i < C.op.size(); ++i)
    if ((C.op[i] >> 1) == f) L.push_back((int)i);
  const int N = (int)L.size();
  const double beta = mc->beta;
  const FlavorDet& D = C.fl[f];
  if (u[0] < 0.5) {
    double t_c, t_a;
    if (N == 0) {
      t_c = u[2] * beta;
      t_a = u[3] * beta;
      m.q = beta * beta;
    } else {
      const int k = std::min(N - 1, (int)(u[2] * N));
      const int o = L[k], nx = L[(k + 1) % N];
      double d = C.tau[nx] - C.tau[o];
      if (d <= 0.0) d += beta;
      const double x1 = u[3] * d, x2 = u[5] * d;
      if (x1 == x2) return;
      double t_lo = C.tau[o] + std::min(x1, x2), t_hi = C.tau[o] + std::max(x1, x2);
      if (t_lo >= beta) t_lo -= beta;
      if (t_hi >= beta) t_hi -= beta;
      const bool first_is_creator = (C.op[o] & 1) == 0;  // after an annihilator the flavor is empty
      t_c = first_is_creator ? t_lo : t_hi;
      t_a = first_is_creator ? t_hi : t_lo;
      m.q = (double)N * d * d / (2.0 * (N + 2));
    }
    if (t_c == t_a || time_taken(C, t_c) || time_taken(C, t_a)) return;
    if ((int)C.op.size() + 2 > ctr::kMaxOps) return;
    m.tc = t_c;
    m.ta = t_a;
    // Schur complement of the bordered block: ratio = S - R inv Q
    const int kk = D.k;
    m.v.assign(kk, 0.0);
    m.w.assign(kk, 0.0);
    std::vector<double> Q(kk), R(kk);
    for (int r = 0; r < kk; ++r) Q[r] = delta(mc, f, D.tc[r] - t_a);
    for (int s = 0; s < kk; ++s) R[s] = delta(mc, f, t_c - D.ta[s]);
    for (int s = 0; s < kk; ++s) {
      double acc = 0.0;
      for (int r = 0; r < kk; ++r) acc += D.inv[(size_t)s * kk + r] * Q[r];
      m.v[s] = acc;
    }
    for (int r = 0; r < kk; ++r) {
      double acc = 0.0;
      for (int s = 0; s < kk; ++s) acc += R[s] * D.inv[(size_t)s * kk + r];
      m.w[r] = acc;
    }
    double ratio = delta(mc, f, t_c - t_a);
    for (int s = 0; s < kk; ++s) ratio -= R[s] * m.v[s];
    m.ratio = ratio;
    m.kind = 0;
    return;
  }
  if (N == 0) return;
  const int k = std::min(N - 1, (int)(u[2] * N));
  const int o = L[k], nx = L[(k + 1) % N];
  if (N == 2) {
    m.q = 1.0 / (beta * beta);
  } else {
    const int prev = L[(k - 1 + N) % N], after = L[(k + 2) % N];
    double d = C.tau[after] - C.tau[prev];
    if (d <= 0.0) d += beta;
    m.q = 2.0 * N / ((N - 2) * d * d);
  }
  m.ic = (C.op[o] & 1) ? o : nx;
  m.ia = (C.op[o] & 1) ? nx : o;
  m.rc = (int)(std::find(D.tc.begin(), D.tc.end(), C.tau[m.ic]) - D.tc.begin());
  m.ra = (int)(std::find(D.ta.begin(), D.ta.end(), C.tau[m.ia]) - D.ta.begin());
  m.ratio = D.inv[(size_t)m.ra * D.k + m.rc];
  m.kind = 1;
}

// The proposal's operator list, written to tau/op (room for its length).
void proposed_string_to(const Chain& C, const Move& m, int f, double* tau, int32_t* op) {
  size_t k = 0;
  if (m.kind == 0) {
    const double t1 = std::min(m.tc, m.ta), t2 = std::max(m.tc, m.ta);
    const int32_t o1 = t1 == m.tc ? 2 * f + 1 : 2 * f, o2 = t1 == m.tc ? 2 * f : 2 * f + 1;
    size_t i = 0;
    for (; i < C.tau.size() && C.tau[i] < t1; ++i, ++k) {
      tau[k] = C.tau[i];
      op[k] = C.op[i];
    }
    tau[k] = t1;
    op[k++] = o1;
    for (; i < C.tau.size() && C.tau[i] < t2; ++i, ++k) {
      tau[k] = C.tau[i];
      op[k] = C.op[i];
    }
    tau[k] = t2;
    op[k++] = o2;
    for (; i < C.tau.size(); ++i, ++k) {
      tau[k] = C.tau[i];
      op[k] = C.op[i];
    }
  } else {
    for (size_t i = 0; i < C.tau.size(); ++i)
      if ((int)i != m.ic && (int)i != m.ia) {
        tau[k] = C.tau[i];
        op[k++] = C.op[i];
      }
  }
}

// The proposal's operator list.
void proposed_string(const Chain& C, const Move& m, int f, std::vector<double>& tau, std::vector<int32_t>& op) {
  if (m.kind == 0) {
    const double t1 = std::min(m.tc, m.ta), t2 = std::max(m.tc, m.ta);
    const int32_t o1 = t1 == m.tc ? 2 * f + 1 : 2 * f, o2 = t1 == m.tc ? 2 * f : 2 * f + 1;
    size_t i = 0;
    for (; i < C.tau.size() && C.tau[i] < t1; ++i) {
      tau.push_back(C.tau[i]);
      op.push_back(C.op[i]);
    }
    tau.push_back(t1);
    op.push_back(o1);
    for (; i < C.tau.size() && C.tau[i] < t2; ++i) {
      tau.push_back(C.tau[i]);
      op.push_back(C.op[i]);
    }
    tau.push_back(t2);
    op.push_back(o2);
    for (; i < C.tau.size(); ++i) {
      tau.push_back(C.tau[i]);
      op.push_back(C.op[i]);
    }
  } else {
    for (size_t i = 0; i < C.tau.size(); ++i)
      if ((int)i != m.ic && (int)i != m.ia) {
        tau.push_back(C.tau[i]);
        op.push_back(C.op[i]);
      }
  }
}

// Accepted move: update the flavor block's inverse (bordering or deletion
// formulas), refreshed from scratch every rebuild_every updates.
void commit(const ctr_mc* mc, Chain& C, const Move& m, double la_loc_new) {
  FlavorDet& D = C.fl[m.f];
  const int k = D.k;
  if (m.kind == 0) {
    const double st = 1.0 / m.ratio;
    std::vector<double> ni((size_t)(k + 1) * (k + 1));
    for (int s = 0; s < k; ++s) {
      for (int r = 0; r < k; ++r) ni[(size_t)s * (k + 1) + r] = D.inv[(size_t)s * k + r] + m.v[s] * st * m.w[r];
      ni[(size_t)s * (k + 1) + k] = -m.v[s] * st;
    }
    for (int r = 0; r < k; ++r) ni[(size_t)k * (k + 1) + r] = -st * m.w[r];
    ni[(size_t)k * (k + 1) + k] = st;
    D.inv.swap(ni);
    D.tc.push_back(m.tc);
    D.ta.push_back(m.ta);
    D.k = k + 1;
  } else {
    const int i = m.rc, j = m.ra;
    const double p = D.inv[(size_t)j * k + i];
    std::vector<double> col(k), row(k);
    for (int s = 0; s < k; ++s) col[s] = D.inv[(size_t)s * k + i];
    for (int r = 0; r < k; ++r) row[r] = D.inv[(size_t)j * k + r];
    for (int s = 0; s < k; ++s)
      for (int r = 0; r < k; ++r) D.inv[(size_t)s * k + r] -= col[s] * row[r] / p;
    // delete column i (creator) and row j (annihilator): the last ones move into their place
    const int last = k - 1;
    for (int s = 0; s < k; ++s) D.inv[(size_t)s * k + i] = D.inv[(size_t)s * k + last];
    for (int r = 0; r < k; ++r) D.inv[(size_t)j * k + r] = D.inv[(size_t)last * k + r];
    std::vector<double> ni((size_t)last * last);
    for (int s = 0; s < last; ++s)
      for (int r = 0; r < last; ++r) ni[(size_t)s * last + r] = D.inv[(size_t)s * k + r];
    D.inv.swap(ni);
    D.tc[i] = D.tc[last];
    D.ta[j] = D.ta[last];
    D.tc.pop_back();
    D.ta.pop_back();
    D.k = last;
  }
  D.ld += std::log(std::fabs(m.ratio));
  C.la_loc = la_loc_new;
  std::vector<double> nt;
  std::vector<int32_t> no;
  proposed_string(C, m, m.f, nt, no);
  C.tau.swap(nt);
  C.op.swap(no);
  if (++D.updates >= mc->rebuild_every && D.k > 0) {
    double ld = 0.0;
    if (rebuild(mc, m.f, D, &ld)) D.ld = ld;  // a singular refresh keeps the updated inverse
  }
  C.la_hyb = 0.0;
  for (const FlavorDet& E : C.fl) C.la_hyb += E.ld;
}

double log_abs_value(const ctr_value& v) {
  const double a = std::hypot(v.re, v.im);
  return a > 0.0 ? std::log(a) + v.log_scale : -INFINITY;
}

}  // namespace

extern "C" {

ctr_status ctr_mc_create(ctr_ctx* ctx, const ctr_mc_opts* opts, ctr_mc** out) {
  if (!out) return CTR_ERR_ARG;
  *out = nullptr;
  if (!ctx || !opts || opts->n_chains < 1 || opts->n_bath < 0 || opts->rebuild_every < 0 ||
      (opts->full_traces != 0 && opts->full_traces != 1) ||
      (opts->n_bath > 0 && (!opts->bath_eps || !opts->bath_v)))
    return CTR_ERR_ARG;
  if (!ctr::context_loaded(ctx)) return CTR_ERR_STATE;
  ctr_mc* mc = new ctr_mc();
  mc->ctx = ctx;
  mc->nf = ctr::context_nops(ctx) / 2;
  mc->nb = opts->n_bath;
  mc->beta = ctr::context_beta(ctx);
  mc->rebuild_every = opts->rebuild_every ? opts->rebuild_every : 64;
  mc->full = opts->full_traces == 1;
  mc->eps.assign(opts->bath_eps, opts->bath_eps + (size_t)mc->nf * mc->nb);
  mc->vv.assign(opts->bath_v, opts->bath_v + (size_t)mc->nf * mc->nb);
  for (size_t i = 0; i < mc->eps.size(); ++i)
    if (!std::isfinite(mc->eps[i]) || !std::isfinite(mc->vv[i])) {
      delete mc;
      return CTR_ERR_ARG;
    }
  // every chain starts at order zero: w_loc = Z, w_hyb = 1
  ctr_value z{};
  const ctr_status s = ctr_trace(ctx, 0, nullptr, nullptr, nullptr, &z);
  if (s != CTR_OK) {
    delete mc;
    return s;
  }
  Chain c0;
  c0.fl.assign(mc->nf, FlavorDet{});
  c0.la_loc = log_abs_value(z);
  mc->chains.assign(opts->n_chains, c0);
  mc->moves.resize(opts->n_chains);
  mc->thr_c.assign(opts->n_chains, 0.0);
  mc->len_c.assign(opts->n_chains, -1);
  mc->slot_c.assign(opts->n_chains, -1);
  mc->acc_c.assign(opts->n_chains, 0);
  // host workers: the hardware threads, at most 16, the caller being one of them
  const int hw = (int)std::thread::hardware_concurrency();
  mc->pool.reset(new Pool(std::max(0, std::min(hw, 16) - 1)));
  *out = mc;
  return CTR_OK;
}

ctr_status ctr_mc_set_config(ctr_mc* mc, int32_t chain, int32_t n_ops, const double* tau, const int32_t* op) {
  if (!mc || chain < 0 || chain >= (int)mc->chains.size() || n_ops < 0 || n_ops > ctr::kMaxOps ||
      (n_ops > 0 && (!tau || !op)))
    return CTR_ERR_ARG;
  for (int i = 0; i < n_ops; ++i) {
    if (!(tau[i] >= 0.0 && tau[i] < mc->beta) || op[i] < 0 || op[i] >= 2 * mc->nf) return CTR_ERR_RANGE;
    if (i > 0 && !(tau[i] > tau[i - 1])) return CTR_ERR_UNSORTED;
  }
  // the pair moves keep every flavor alternating between creators and annihilators
  for (int f = 0; f < mc->nf; ++f) {
    int first = -1, last = -1;
    for (int i = 0; i < n_ops; ++i) {
      if ((op[i] >> 1) != f) continue;
      if (last >= 0 && (op[i] & 1) == last) return CTR_ERR_ARG;
      if (first < 0) first = op[i] & 1;
      last = op[i] & 1;
    }
    if (first >= 0 && first == last) return CTR_ERR_ARG;
  }
  Chain C;
  C.tau.assign(tau, tau + n_ops);
  C.op.assign(op, op + n_ops);
  if (!build_hyb(mc, C)) return CTR_ERR_ARG;  // unbalanced flavor or singular hybridisation block
  ctr_value v{};
  const ctr_status s = ctr_trace(mc->ctx, n_ops, tau, op, nullptr, &v);
  if (s != CTR_OK) return s;
  C.la_loc = log_abs_value(v);
  if (!std::isfinite(C.la_loc)) return CTR_ERR_ARG;  // zero local weight
  mc->chains[chain] = std::move(C);
  return CTR_OK;
}

ctr_status ctr_mc_step(ctr_mc* mc, const double* u, int32_t* decision) {
  if (!mc || !u) return CTR_ERR_ARG;
  using Clock = std::chrono::steady_clock;
  const Clock::time_point t0 = Clock::now();
  const int n = (int)mc->chains.size();
  for (long long i = 0; i < 6LL * n; ++i)
    if (!(u[i] >= 0.0 && u[i] < 1.0)) return CTR_ERR_RANGE;
  // pass 1, per chain: draw the move, its hybridisation ratio and its trace threshold
  mc->pool->run(n, [&](int c) {
    const Chain& C = mc->chains[c];
    Move& m = mc->moves[c];
    const double* uc = u + 6LL * c;
    propose(mc, C, uc, m);
    mc->len_c[c] = -1;
    mc->acc_c[c] = 0;
    if (m.kind < 0 || !(std::fabs(m.ratio) > 0.0) || !std::isfinite(m.ratio)) return;  // no trace needed
    // accept iff q |ratio| |w_loc'| >= u4 |w_loc|: the rest of the ratio goes into the trace threshold
    const double log_r = uc[4] > 0.0 ? std::log(uc[4]) : -INFINITY;
    mc->thr_c[c] = log_r + C.la_loc - std::log(m.q) - std::log(std::fabs(m.ratio));
    mc->len_c[c] = (int64_t)C.op.size() + (m.kind == 0 ? 2 : -2);
  });
  // batch layout in chain order
  mc->offs.assign(1, 0);
  mc->thr.clear();
  mc->bchain.clear();
  for (int c = 0; c < n; ++c) {
    if (decision) decision[c] = mc->moves[c].kind < 0 ? -1 : 0;
    if (mc->moves[c].kind >= 0) mc->n_proposed += 1;
    mc->slot_c[c] = -1;
    if (mc->len_c[c] < 0) continue;
    mc->slot_c[c] = (int32_t)mc->bchain.size();
    mc->bchain.push_back(c);
    mc->thr.push_back(mc->thr_c[c]);
    mc->offs.push_back(mc->offs.back() + mc->len_c[c]);
  }
  const int nb = (int)mc->bchain.size();
  mc->btau.resize((size_t)std::max<int64_t>(mc->offs.back(), 1));
  mc->bop.resize((size_t)std::max<int64_t>(mc->offs.back(), 1));
  // pass 2, per proposal: its operator list into the batch
  mc->pool->run(nb, [&](int b) {
    const int c = mc->bchain[b];
    const Move& m = mc->moves[c];
    proposed_string_to(mc->chains[c], m, m.f, mc->btau.data() + mc->offs[b], mc->bop.data() + mc->offs[b]);
  });
  mc->out.assign(nb, ctr_value{});
  const Clock::time_point t1 = Clock::now();
  if (nb > 0) {
    const ctr_status s =
        mc->full ? ctr_trace_batch(mc->ctx, nb, mc->offs.data(), mc->btau.data(), mc->bop.data(), nullptr,
                                   mc->out.data())
                 : ctr_trace_lazy_batch(mc->ctx, nb, mc->offs.data(), mc->btau.data(), mc->bop.data(),
                                        mc->thr.data(), nullptr, mc->out.data());
    if (s != CTR_OK) return s;
  }
  const Clock::time_point t2 = Clock::now();
  // pass 3, per proposal: the decision and the update of an accepted chain
  mc->pool->run(nb, [&](int b) {
    const int c = mc->bchain[b];
    const ctr_value& v = mc->out[b];
    if (v.flags & CTR_FLAG_REJECTED) return;
    const double la = log_abs_value(v);
    if (!(la >= mc->thr[b]) || !std::isfinite(la)) return;
    commit(mc, mc->chains[c], mc->moves[c], la);
    mc->acc_c[c] = 1;
  });
  for (int b = 0; b < nb; ++b) {
    const int c = mc->bchain[b];
    if (mc->out[b].flags & CTR_FLAG_REJECTED) mc->n_lazy_rejected += 1;
    if (mc->acc_c[c]) {
      mc->n_accepted += 1;
      if (decision) decision[c] = 1;
    }
  }
  mc->n_steps += 1;
  const Clock::time_point t3 = Clock::now();
  mc->host_ms += std::chrono::duration<double, std::milli>((t1 - t0) + (t3 - t2)).count();
  mc->trace_ms += std::chrono::duration<double, std::milli>(t2 - t1).count();
  return CTR_OK;
}

ctr_status ctr_mc_config(const ctr_mc* mc, int32_t chain, int32_t cap, double* tau, int32_t* op, int32_t* n_ops,
                         double* log_w) {
  if (!mc || chain < 0 || chain >= (int)mc->chains.size() || !n_ops || cap < 0) return CTR_ERR_ARG;
  const Chain& C = mc->chains[chain];
  *n_ops = (int32_t)C.op.size();
  if ((int)C.op.size() > cap) return CTR_ERR_ARG;
  if (!C.op.empty() && (!tau || !op)) return CTR_ERR_ARG;
  std::copy(C.tau.begin(), C.tau.end(), tau);
  std::copy(C.op.begin(), C.op.end(), op);
  if (log_w) {
    log_w[0] = C.la_loc;
    log_w[1] = C.la_hyb;
  }
  return CTR_OK;
}

ctr_status ctr_mc_stats(const ctr_mc* mc, int64_t* n_steps, int64_t* n_proposed, int64_t* n_lazy_rejected,
                        int64_t* n_accepted) {
  if (!mc || !n_steps || !n_proposed || !n_lazy_rejected || !n_accepted) return CTR_ERR_ARG;
  *n_steps = mc->n_steps;
  *n_proposed = mc->n_proposed;
  *n_lazy_rejected = mc->n_lazy_rejected;
  *n_accepted = mc->n_accepted;
  return CTR_OK;
}

ctr_status ctr_mc_timing(const ctr_mc* mc, double* host_ms, double* trace_ms) {
  if (!mc || !host_ms || !trace_ms) return CTR_ERR_ARG;
  *host_ms = mc->host_ms;
  *trace_ms = mc->trace_ms;
  return CTR_OK;
}

void ctr_mc_destroy(ctr_mc* mc) { delete mc; }

}  // extern "C"
