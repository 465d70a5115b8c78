// Internal data structures shared by the host side of the C ABI and the
// gfx950 kernels.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ctrace.h"

namespace ctr {

constexpr int kPanel = 16;        // columns of the carried matrix per work item (one MFMA tile)
constexpr int kMaxOps = 512;      // operators per configuration (held in LDS by the kernels)
constexpr int kPlanThreads = 256;

inline int pad16(int x) { return (x + 15) & ~15; }
inline int pad4(int x) { return (x + 3) & ~3; }

// Impurity as resident in the arena (all pointers are device addresses).
struct DevImp {
  int n_sec;
  int nops;          // 2 * n_flavors
  int is_complex;
  int xrows;         // pad16(largest sector dimension)
  int next_lds;      // 1 if the chain kernel keeps the sector map in LDS
  int pad_;
  double beta;
  double E0;         // global lowest eigenvalue
  const int* dim;            // [n_sec]
  const int* next;           // [n_sec * nops]
  const long long* boff;     // [n_sec * nops] offset (in doubles) of block (q, op) in pool, -1 if none
  const double* emin;        // [n_sec] lowest eigenvalue of every sector
  const int* eoff;           // [n_sec] offset of the sector's energies in esh
  const double* esh;         // energies minus the sector's lowest one, zero padded to pad16(dim)
  const double* lognorm;     // [n_sec * nops] log spectral norm of every block (0 when unknown)
  const long long* roff;     // [n_sec * nops] offset of the block's row exponents in rexp
  const short* rexp;         // per block and padded row: e with max_k |F[m][k]| < 2^e (FP32-split scaling)
  const double* pool;        // operator blocks
  // [n_sec * nops * 8] nonzero 16 x 4 tiles of blocks of at most 128 x 128: word 8 * (q * nops + op) + t
  // has bit c set iff rows 16 t .. 16 t + 15, columns 4 c .. 4 c + 3 hold a nonzero (either plane);
  // all bits set for larger blocks
  const unsigned int* tmask;
};
// Block (q, op) with d_out = dim[next[q][op]], d_in = dim[q] is stored column-major:
// element (row m, column k) at pool[boff + k * pad16(d_out) + m], columns padded to pad4(d_in),
// zero padding; a complex block keeps its imaginary plane right after the real one.

// One (configuration, start sector) string after the walk.
struct StrRec {
  int q_start;     // sector at the rotated start position
  int jstar;       // rotated start position (index of the first operator applied)
  int width;       // dimension of the start sector (columns of the carried matrix)
  int n_panels;    // ceil(width / panel width) if the string survives, else 0
  int loc_off;     // panel offset of this string inside its configuration
  int pad;
  double L;        // sum over positions of dt * (lowest energy of the sector - E0)
  double logB;     // log of the lazy bound of this string (without the -beta*E0 part)
  unsigned long long u_full;  // lazy traces: initial bound of a full panel, in threshold units
  unsigned long long u_last;  // same for the last (possibly narrower) panel
};

// Lazy traces keep the running bound sum of a configuration exactly, in
// integer units of 2^-kLazyUnitBits times its threshold: a panel bound b
// counts ceil(b / unit) (at most kLazyCap), and the configuration is
// rejected once the sum is below 2^kLazyUnitBits.  Integer sums do not
// cancel, whatever the ratio of the threshold to the initial bound.
constexpr int kLazyUnitBits = 30;
constexpr int kLazyCapBits = 40;

struct PanelRes {
  double re, im;   // mantissa
  double e2;       // power-of-two exponent: panel contribution = (re + i im) * 2^e2 * exp(-L)
};

struct BatchArgs {
  int n_cfg;
  int panel;                 // columns per work item (16 block kernel, 8 wavefront kernel)
  const long long* offsets;  // [n_cfg + 1] absolute indices into tau / op
  const double* tau;
  const int* op;
  const double* log_thr;     // [n_cfg] lazy thresholds or nullptr
  StrRec* rec;               // [n_cfg * n_sec]
  int* cfg_cnt;              // [n_cfg] panels per configuration
  int* cfg_flags;            // [n_cfg]
  int* cfg_nstr;             // [n_cfg]
  double* cfg_logB;          // [n_cfg]
  long long* cfg_off;        // [n_cfg + 1]
  PanelRes* res;             // [total panels]
  unsigned int* counter;     // persistent-kernel work counter
  ctr_value* out;            // [n_cfg]
  // lazy traces (log_thr != nullptr)
  double* cfg_lthr;                  // [n_cfg] log threshold + beta*E0 (units of the string bounds)
  unsigned long long* cfg_bsum;      // [n_cfg] running sum of panel bounds in threshold units
  int* cfg_rej;                      // [n_cfg] 1 once the bound sum fell below the threshold
};

// Block-grouped evaluation (ctrace_group.hip): every surviving string is one
// chain over its start sector's columns; all strings advance one operator per
// round and the strings at the same block in a round share one wide product.
// Round r >= 1, group key k: block q*nops+op (k < NB) or, at a string's last
// operator, NB + block (the close); NB = n_sec * nops, NK = 2 * NB.
struct GroupArgs {
  long long S;                 // surviving strings of the batch
  long long T;                 // columns (sum of string widths)
  int R;                       // rounds (largest operator count)
  int cw_step, cw_close;       // columns per work item (products, closes)
  long long CS;                // column-steps: sum over strings of width * (operators - 1)
  long long NI;                // bound on the work items of all rounds
  int* s_cfg;                  // [S] configuration of the string
  int* s_rec;                  // [S] its record (start-sector index) in the configuration
  int* s_width;                // [S] columns of the string
  int* s_n;                    // [S] operators of its configuration
  long long* s_colbase;        // [S] first column of the string
  long long* info;             // [5] S, T, R, CS, NI (device copy, read back by the host)
  int* hist;                   // [R][NK] strings per group
  int* hcols;                  // [R][NK] columns per group
  int* cursor;                 // [R][NK] scatter cursors
  int* gstart;                 // [R][NK+1] first position of every group in `sorted`
  int* istart;                 // [R][NK+1] first work item of every group
  int* n_items;                // [R]
  unsigned int* counters;      // [R][kGroupCounters * 32] persistent-kernel work counters, one per 128-byte line
  int* sorted;                 // [R][S] strings in group order
  int* colpref;                // [R][S] first column (round-relative) of every sorted string
  long long* rcols;            // [R] columns of round r
  long long* rcoloff;          // [R] first column-step of round r in colg / colaux
  long long* ritemoff;         // [R] first work item of round r in item_key
  int* item_key;               // [NI] group of every work item
  int* colg;                   // [CS] column-steps in group order: global column
  double* colaux;              // [CS] gap in front of the next operator (products) or the
                               //      column's index inside its start sector (closes)
  double* X[2];                // carried matrices, ping-pong: column g at g * xrows (imaginary plane at + T * xrows)
  int* colexp;                 // [T] accumulated power of two of every column
  PanelRes* colres;            // [T] closed column values
  // Sectors beyond one workgroup's register tile: product items cover rchunk
  // rows of the block (0 = all rows).  The per-column power of two of a round
  // is then a device-wide integer maximum over the row chunks, kept pending in
  // epend[(r + 1) % 3] (unscaled values stored) and applied by the loads of
  // round r + 1; round r resets epend[(r + 2) % 3] for the rounds after.
  int rchunk;
  int* epend;                  // [3][T] pending exponents, kNoExp = none
};
constexpr int kNoExp = -(1 << 20);

// Label histogram of a batch (ctrace_hist.hip), after the combine kernel.
// The values of string (c, q0) with record R are vals[colbase[cfg_off[c] +
// R.loc_off] + j], j < R.width (grouped rounds: one value per column), or
// vals[cfg_off[c] + R.loc_off + p], p < R.n_panels (per-string kernels:
// one value per panel), as the combine kernels read them.
struct HistArgs {
  const int* label;          // [n_sec] label of every sector, 0 .. n_labels-1
  int n_labels;
  const PanelRes* vals;
  const long long* colbase;  // grouped rounds: first column of every string; nullptr otherwise
  double* hist;              // [n_cfg][n_labels] complex (re, im)
};

// Density-matrix estimator of a batch (ctrace_rdm.hip), after the traces are known.
constexpr int kRdmMaxRows = 1024;  // largest sector the estimator handles
struct RdmArgs {
  double* buf;                 // per-workgroup buffers, per_wg doubles each
  size_t per_wg;
  int slots;                   // stored forward products per string: the batch's largest operator count (>= 1)
  const double* w;             // [n_cfg][2] trace mantissas (the combine kernel's output)
  const double* wlog;          // [n_cfg] their log scale + beta E0 (the units of the string shifts L)
  const double* weight;        // [n_cfg][2] caller weights
  double* rho;                 // [sum_q dim_q^2][2] output, accumulated with atomic adds
  const long long* rho_off;    // [n_sec] first entry of every sector's block
};

// Launchers (ctrace_kernels.hip, ctrace_group.hip, ctrace_hist.hip, ctrace_rdm.hip).  All enqueue on `stream`.
hipError_t launch_plan(const DevImp& imp, const BatchArgs& b, hipStream_t stream);
hipError_t launch_scan(const BatchArgs& b, hipStream_t stream);
// split: 0 = FP64 block products, 6 or 7 = FP32-split with that many 8-bit slices
hipError_t launch_chain(const DevImp& imp, const BatchArgs& b, int split, int grid, hipStream_t stream);
hipError_t launch_combine(const DevImp& imp, const BatchArgs& b, hipStream_t stream);
hipError_t launch_hist(const DevImp& imp, const BatchArgs& b, const HistArgs& h, hipStream_t stream);
// LDS bytes and persistent grid size of the chain kernel for this impurity; grid 0 = unsupported.
int chain_grid(const DevImp& imp, int device, int split, size_t* lds_bytes);
size_t chain_lds_bytes(const DevImp& imp);
int chain_max_rows(int is_complex);
// Wavefront-per-panel chain kernel (sectors of at most 128 states); grid 0 = not applicable.
int wave_grid(const DevImp& imp, int device, size_t* lds_bytes, bool lazy = false);
hipError_t launch_chain_wave(const DevImp& imp, const BatchArgs& b, int grid, hipStream_t stream);
constexpr int kWavePanelHost = 8;
// Streaming chain kernel (any sector size; X in per-workgroup global buffers).
int big_grid(const DevImp& imp, int device, size_t* lds_bytes);
size_t big_xbuf_doubles(const DevImp& imp, int grid);
hipError_t launch_chain_big(const DevImp& imp, const BatchArgs& b, double* xbuf, int grid, hipStream_t stream);
// Block-grouped path; grid 0 = not applicable.  rchunk_out (may be null) gets
// the rows per product item of the chosen shape (0 = every row in one item).
// alt = 1: the alternative tile shape (grid 0 when there is none for this impurity).
// split: 0 FP64 products, 6 or 7 the FP32-split row-chunked items (alt 2 only).
int group_grid(const DevImp& imp, int device, int alt, int* cw_step, int* rchunk_out = nullptr, int split = 0);
hipError_t launch_group_prepare(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, long long max_strings,
                                hipStream_t stream);
hipError_t launch_group_schedule(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, hipStream_t stream);
hipError_t launch_group_round(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, int r, int grid, int alt,
                              int split, hipStream_t stream);
hipError_t launch_group_combine(const DevImp& imp, const BatchArgs& b, const GroupArgs& g, hipStream_t stream);
// Kernel-node parameters of round launches for a HIP graph (args: {&imp, &b, &g, &r}, kept alive by the caller
// until the node is added).
hipError_t group_round_node(const DevImp& imp, const GroupArgs& g, int grid, int alt, int split, void** args,
                            hipKernelNodeParams* p);
size_t rdm_buffer_doubles(const DevImp& imp, int slots);
int rdm_grid(int device);
hipError_t launch_rdm(const DevImp& imp, const BatchArgs& b, const RdmArgs& d, int grid, hipStream_t stream);
// Peak-rate probe (ctrace_probe.hip): out[0..4] = FP64 16x16x4 and 4x4x4 MFMA and FP32 16x16x4
// MFMA TFLOP/s, clock (MHz), compute units.  sink: 256 doubles of device memory.
hipError_t probe_peaks(int device, hipStream_t stream, double* sink, double* out);
// Context queries for the serving layer (ctrace_host.cpp); read-only after ctr_set_impurity.
bool context_loaded(const ctr_ctx* ctx);
double context_beta(const ctr_ctx* ctx);
int context_nops(const ctr_ctx* ctx);
size_t context_free_scratch(const ctr_ctx* ctx);          // arena bytes not held by the impurity
// Arena bytes one configuration occupies in a batch call: per-call scratch, and with the grouped
// rounds the carried matrices of its surviving strings (host walk of the sector map).
size_t request_scratch_bytes(const ctr_ctx* ctx, long long n_ops, const int32_t* op);
// Block-product flops of one configuration (its surviving strings at their narrowest width; host walk).
double request_flops(const ctr_ctx* ctx, long long n_ops, const int32_t* op);
// Fraction in (0, 1] of every persistent grid the context launches (1 = the whole device).
void context_set_grid_share(ctr_ctx* ctx, double share);

constexpr int kGroupCloseCols = 64;
// Work items of a round are spread over this many counters (item i belongs to
// counter i % kGroupCounters): one device-scope atomic address serialises.
constexpr int kGroupCounters = 64;
constexpr int kGroupPanel = 1 << 24;  // plan panel width in grouped mode: one panel per string

}  // namespace ctr
