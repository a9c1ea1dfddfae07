// Internal declarations of libddg: handle layout, error plumbing, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/ddg.h"
#include "device_util.hpp"

namespace ddg {

// ---------------------------------------------------------------------------
// Errors

struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string& msg);
void clear_error();

#define DDG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      throw ::ddg::Error{_e == hipErrorOutOfMemory ? DDG_ERR_OOM : DDG_ERR_HIP,    \
                         std::string(#call) + ": " + hipGetErrorString(_e)};       \
    }                                                                              \
  } while (0)

#define DDG_REQUIRE(cond, code, text)                                              \
  do {                                                                             \
    if (!(cond)) throw ::ddg::Error{(code), (text)};                               \
  } while (0)

// ---------------------------------------------------------------------------
// Device buffer (owning)

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t nbytes) {
    release();
    if (nbytes == 0) nbytes = 16;
    DDG_HIP(hipMalloc(&p, nbytes));
    bytes = nbytes;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
  template <class T> void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size() * sizeof(T));
    if (!v.empty()) DDG_HIP(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
  }
};

// ---------------------------------------------------------------------------
// Host symbolic structure (integers only; no floating-point arithmetic of the method)

struct Symbolic {
  int64_t n = 0, nnz = 0;
  int32_t n_parts = 0, overlap = 0;
  std::vector<int64_t> own_ptr;      // n_parts+1, non-overlapping sets (ascending)
  std::vector<int32_t> own_idx;      // n
  std::vector<int64_t> set_ptr;      // n_parts+1, expanded sets
  std::vector<int32_t> set_idx;      // sum |set|
  std::vector<int32_t> colour;       // n_parts
  int32_t n_colours = 0;
  std::vector<int32_t> colour_ptr;   // n_colours+1 into colour_subs
  std::vector<int32_t> colour_subs;  // subdomains grouped by colour, ascending id
  std::vector<int32_t> nbr_ptr;      // n_parts+1, coupled subdomains (incl. self), ascending
  std::vector<int32_t> nbr_idx;
  std::vector<int32_t> conf_ptr;     // n_parts+1, conflicting subdomains (set meets the other's
  std::vector<int32_t> conf_idx;     //   neighbourhood), ascending, self excluded
  // blocks of the local factors
  std::vector<int32_t> sub_blk_ptr;  // n_parts+1 into block arrays
  std::vector<int32_t> blk_start;    // first local row of each block
  std::vector<int32_t> blk_size;     // rows of each block
  std::vector<int64_t> blk_foff;     // element offset of each block's tiles in the factor array
  std::vector<int32_t> sub_mid;      // middle level m of each subdomain's twisted factorisation
  int64_t fac_elems = 0;
  int32_t tile = 64;
  int32_t max_set = 0, max_blk = 0, max_blocks = 0, max_own = 0;
  // local couplings, per local row r (global row id = set_ptr[i] + j):
  //   lower (to the previous level) and upper (to the next level) in ELL form with
  //   cl / cu slots per row (col = -1 marks an empty slot), same-level entries in CSR form.
  int32_t cl = 0, cu = 0;
  std::vector<int32_t> lo_col, up_col;           // rows * cl, rows * cu: local column or -1
  std::vector<int64_t> lo_pos, up_pos;           // position in the global CSR value array (or -1)
  std::vector<int64_t> in_ptr;                   // sum|set|+1
  std::vector<int32_t> in_col;
  std::vector<int64_t> in_pos;
  // The same lower/upper couplings in the sweep's sliced layout, built when some row
  // has more than kCplRegs couplings in a direction: every level is cut into slices
  // of 64 consecutive rows; a slice stores its entries column by column (entry q of
  // its row at lane l sits at off[slice] + 64 q + l), padded to the slice's longest
  // row with value 0 and the row's own local index as column (lanes past the end of
  // the block: column 0, never read).  The values are refreshed from the ELL arrays.
  bool sliced = false;
  std::vector<int32_t> blk_slice;                // n_blocks+1: first slice of each block
  int32_t max_sub_slices = 0;                    // most slices of one subdomain
  std::vector<int64_t> sl_row;                   // per slice: global set row of its lane 0
  std::vector<int32_t> sl_rows;                  // per slice: rows of the block it holds (<= 64)
  std::vector<int64_t> sl_lo_off, sl_up_off;     // n_slices+1 entry offsets
  std::vector<int32_t> sl_lo_col, sl_up_col;     // local column of each entry
};

// Most generating vectors per system (degree 10 in 2D has 66); the coarse kernels
// keep per-thread column arrays of 32 entries, or of kMaxGen when k > 32.
constexpr int kMaxGen = 80;
// grouped sweep: workgroups per chain at most (default, and the most DDG_SWEEP_GROUPS
// may ask for), narrowest split level in rounds
constexpr int kSweepGroupsMax = 4;
constexpr int kSweepGroupsCap = 8;
constexpr int kSweepSplitRounds = 4;
inline int32_t kslots(int32_t k) { return k <= 32 ? 32 : kMaxGen; }

// Couplings per row and direction that the sweep keeps in registers; wider rows use
// the sliced layout.
constexpr int kCplRegs = 2;

// Builds every integer structure; throws Error on malformed input.
void build_symbolic(Symbolic& S, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                    const int32_t* part, int32_t n_parts, int32_t overlap, int32_t tile,
                    int32_t block_target);

// Lanes per CSR row in the row-dot kernels for a matrix with nnz entries in n rows:
// about ten entries per lane, one lane for stencil-sized rows.
inline int32_t lanes_per_row(int64_t nnz, int64_t n) {
  const double avg = n > 0 ? (double)nnz / (double)n : 0.0;
  return avg <= 12.0 ? 1 : avg <= 24.0 ? 2 : avg <= 48.0 ? 4 : avg <= 96.0 ? 8 : 16;
}

// Tile layout helpers shared by host and device.
__host__ __device__ inline int32_t tiles_for(int32_t b, int32_t T) {
  int32_t nt = (b + T - 1) / T;
  return nt * (nt + 1) / 2;
}

// ---------------------------------------------------------------------------
// Device-side CG state (one per independent system of the handle)

struct CgState {
  double rho;        // r^T z
  double alpha, beta;
  double pq;
  double rr;         // ||r||^2
  double fnorm;      // ||f||
  double tol2;       // (rtol ||f||)^2
  double true_rr;    // ||f - A x||^2 after the solve
  int32_t done;      // 1 = converged / stopped
  int32_t status;    // ddg_status
  int32_t iters;
  int32_t max_iter;
  uint64_t t_start;  // device real-time counter at the start of the solve
  uint64_t t_done;   // ... when this system stopped
};

// ---------------------------------------------------------------------------
// Buffers that the preconditioner's kernels write and read back within one
// application (nothing in them outlives it): the handle's own, allocated at
// setup, or the library's static scratch (ddg_apply_precond_noalloc).

struct PrecondWs {
  double* bres = nullptr;   // local residuals of one colour's expanded sets (sum |set| values)
  double* rpart = nullptr;  // coarse restriction partials (n_parts x nch x 32)
  double* cy = nullptr;     // coarse right-hand side then solution (2 x nc_pad); zero padding
  double* cpart = nullptr;  // coarse GEMV row and column partials (2 x ntiles x 64)
  double* cref = nullptr;   // coarse refinement residual and correction (2 x nc_pad; refinement only)
};

// ---------------------------------------------------------------------------
// Handle

struct Handle {
  bool host_only = false;   // created by ddg_analyze: symbolic data only
  ddg_options opt{};
  hipStream_t stream = nullptr;
  Symbolic S;
  int32_t k = 0;          // columns of F
  int64_t nc = 0;         // coarse dimension (sum over systems, without padding)
  std::vector<int32_t> kcnt;   // kept columns per subdomain
  std::vector<int64_t> koff;   // coarse offsets (each system's block starts on a multiple of 64)

  // independent systems (a batch): system b owns rows [seg_off[b], seg_off[b+1]) and
  // subdomains [sub_off[b], sub_off[b+1]); its coarse block is rows
  // [cblk_off[b], cblk_off[b] + cblk_n[b]) of the padded coarse vector
  int32_t nb = 1;
  std::vector<int64_t> seg_off;
  std::vector<int32_t> sub_off;
  std::vector<int64_t> cblk_off;     // nb+1, multiples of 64
  std::vector<int32_t> cblk_n;       // nb
  std::vector<int64_t> a0_off;       // nb+1, element offsets of the dense A0 blocks
  std::vector<int64_t> tile_base;    // nb+1, first 64x64 tile of each inverse block
  int64_t nc_pad = 0;                // cblk_off[nb]
  int64_t ntiles = 0;                // tile_base[nb]
  DevBuf sub_inst;                   // int32 per subdomain
  DevBuf cblk_off_d, cblk_n_d, a0_off_d, tile_base_d, tile_inst, trow_inst;
  // CG reduction map: workgroup g covers rows [wg_lo[g], wg_hi[g]) of system wg_seg[g];
  // the partials of system b are [seg_wg_ptr[b], seg_wg_ptr[b+1])
  DevBuf wg_seg, wg_lo, wg_hi, seg_wg_ptr_d;
  std::vector<int32_t> seg_wg_ptr;
  int32_t dev_lds_limit = 65536;
  int32_t lpr = 1;                   // lanes per CSR row in the row-dot kernels (lanes_per_row)
  int32_t rch = 1024;                // own rows per workgroup of the coarse restriction
  int32_t nch = 1;                   // restriction workgroups per subdomain
  DevBuf rpart;                      // restriction partials: n_parts x nch x 32

  // device copies
  DevBuf rowptr, col, val;           // CSR
  DevBuf part, own_ptr, own_idx;
  DevBuf set_ptr, set_idx;
  DevBuf colour_subs;
  DevBuf nbr_ptr, nbr_idx;
  DevBuf sub_blk_ptr, blk_start, blk_size, blk_foff, sub_mid;
  DevBuf lo_col, lo_pos, lo_val;     // ELL lower couplings
  DevBuf up_col, up_pos, up_val;     // ELL upper couplings
  DevBuf in_ptr, in_col, in_pos;
  DevBuf blk_slice, sl_row, sl_rows;                 // sliced couplings (Symbolic::sliced)
  DevBuf sl_lo_off, sl_up_off, sl_lo_col, sl_up_col;
  DevBuf sl_lo_val, sl_up_val;                       // in the sweep's arithmetic type
  DevBuf xch, flags;                 // two-workgroup handoff buffers of the twisted sweep
  DevBuf gx, gcnt;                   // grouped sweep: partial level sums and barrier counts
  // persistent sweep over a task queue (one launch per sweep direction): per
  // direction the subdomains in sweep order and each subdomain's earlier
  // conflicting subdomains; per subdomain a completion count; the queue counter
  bool flow_ok = false;
  DevBuf flow_order[2], flow_dep_ptr[2], flow_dep_idx[2];
  DevBuf flow_done, flow_counter;
  mutable int64_t flow_base = 0;     // queue counter value before the next flow launch
  mutable int32_t flow_seq = 0;      // flow launches so far
  int64_t flow_bytes[2] = {0, 0};    // algorithmic bytes of one flow launch per direction
  DevBuf bres;                       // local residuals of one colour's expanded sets
  // SSOR local smoothing (DDG_LOCAL_SSOR): the local CSR of every A_i over its set
  // rows (per set row t: entries [ss_ptr[t], ss_ptr[t+1]) with local columns and their
  // positions in A's values), the diagonal's position per set row, and per subdomain
  // its local rows sorted by local colour (ss_perm, at the subdomain's set offset) with
  // the colour offsets ss_coff[ss_cptr[i] .. ss_cptr[i+1]] (relative to the set offset)
  bool ssor = false;
  DevBuf ss_ptr, ss_col, ss_pos, ss_val, ss_dpos, ss_diag, ss_perm, ss_cptr, ss_coff;
  std::vector<int64_t> ss_nnz_sub;   // local entries per subdomain (byte accounting)
  // diagonal storage of A (DiaView): possible when every system's entries lie on at
  // most kDiaMax offset pairs; in use while the values are also symmetric bit for bit
  bool dia_possible = false, dia_ok = false;
  int32_t dia_nd = 1;                // upper diagonals stored (most of any system)
  std::vector<DiaSys> dia_sys_h;
  DevBuf dia_sys, dia_diag, dia_up;
  PrecondWs ws;                      // the buffers the preconditioner's kernels use (see PrecondWs)
  // persistent batched solve (DDG_SCHEDULE_PERSISTENT): per (system, colour) subdomain
  // lists, the subdomain offsets of the systems, the initial ring words and per-system
  // states, the per-system states and counts in use, the control words and the ring
  bool persist = false;
  DevBuf ps_ptr, ps_sub, ps_suboff, ps_init, ps_sys0, ps_sys, ps_cnt, ps_ctl, ps_ring, ps_order;
  int32_t ps_ninit = 0;
  int32_t ps_admit = 0;              // systems started at launch (admission order: smallest first)
  int64_t ps_omax = 0;               // most tasks outstanding at once (sum over systems of the largest phase)
  int32_t device = 0;                // HIP device current at setup
  int32_t xch_ld = 0;
  bool twisted_ok = false;
  // grouped sweep (sliced layout): up to grp_max workgroups per chain, levels of at
  // least grp_split rounds split between them; grp_max 1 = off
  int32_t grp_max = 1;
  int32_t grp_split = 0;
  int32_t grp_slots = 0;             // subdomains per launch the buffers hold
  mutable int32_t grp_used = 1;      // largest group size launched so far
  int32_t n_cu = 256;
  // three-level V-cycle: one application of the two-level method of A0 (coarse
  // partition of the subdomains, generating vectors F0 = R0 F, the same overlap)
  // replaces the coarse inverse
  bool three_level = false;
  Handle* inner = nullptr;           // owned: the coarse level's handle
  DevBuf a0_pos;                     // per stored entry of the coarse level's CSR: position in the dense A0
  int64_t apply_bytes = 0;           // algorithmic bytes of one preconditioner application
  DevBuf F;               // n x k column-major (setup input)
  DevBuf Q;               // n x k node-major orthonormal basis (zero-padded)
  DevBuf Qo;              // the same basis in own-row order, 64-row tiles column-major (q_own_at)
  DevBuf qpos;            // n: position of each row in the own-row order
  DevBuf kcnt_d, koff_d;
  DevBuf A0;              // dense coarse blocks, one per system (kept for export)
  DevBuf A0inv_t;         // tiled lower inverses, float64, tile 64
  DevBuf cinv, cwork, cgd;   // coarse inverse: copy of A0 being inverted, recursion workspace, group tables
  struct CoarseGroup {
    int32_t first, count, nfirst;   // items [first, first + count) of the tables, the largest order
    int64_t need;                   // workspace elements per item
  };
  std::vector<CoarseGroup> cinv_groups;   // built once per handle
  int32_t cinv_items = 0;
  // iterative refinement of the coarse solve, y += A0^{-1}_approx (b0 - A0 y), for coarse
  // matrices whose explicit inverse is not accurate to working precision; the step count
  // is chosen at every refactor from the measured ||v - X A0 v|| / ||v||
  int32_t coarse_refine = 0;
  double coarse_inv_err = 0.0;
  // inexact coarse solve (DDG_COARSE_IC_CG): the incomplete Cholesky factor in A0's
  // layout, the inverses of its diagonal blocks, the inner CG's work vectors, the
  // level schedule of the triangular solves (per system levels, rows by level, the
  // subdomain of every coarse row), factorisation marks, inner iteration counts and
  // the subdomain offsets of the systems
  bool ic = false;
  DevBuf icL, icD, icw, ic_sys_lvl, ic_lvl_ptr, ic_lvl_rows, ic_row_sub, ic_mark, ic_it, ic_suboff;
  DevBuf cref, cerr;
  double* h_cerr = nullptr;   // pinned: the power steps' norms of the last measurement
  hipStream_t side = nullptr;  // second stream: the coarse inverse runs beside the local factorisation
  DevBuf fac;             // local factor tiles (storage precision)
  // batched local factorisation: item schedule (built once per handle) and scratch
  struct FacStage {
    int32_t first, count, gj, bmax;
  };
  bool fac_plan_ready = false;
  std::vector<FacStage> fac_stages;
  DevBuf fac_items, fac_off, fac_n, fac_esub, fac_eblk;
  int32_t fac_max_items = 0;
  int64_t fac_wstride = 0;   // per-item workspace of the recursive level inverse
  DevBuf fac_scratch, fac_tm, fac_work;
  DevBuf err_flag;        // int32[4]: setup error (code, subdomain, block, pivot)

  // CG workspace
  DevBuf r, p, q, z, part_sums, cstate;
  DevBuf hist;            // per system: alpha, beta, ||r||^2 histories (max_iter + 1 each)
  bool solved = false;    // a solve has run (the history is valid)
  DevBuf cy, cpart;       // coarse rhs/solution (nc_pad each) and GEMV partials
  DevBuf pinned_state;    // unused placeholder
  CgState* h_state = nullptr;   // pinned host mirror (nb entries)
  int32_t n_partials = 0;

  // info
  ddg_info info{};
  std::vector<ddg_info> sys_info;      // per system, last solve
  int32_t clock_khz = 100000;          // device real-time counter rate
  std::vector<int64_t> colour_bytes;   // algorithmic bytes of one local-solve launch per colour
  std::vector<int64_t> colour_bytes_sys;  // the same per system: [b * 2C + c]
  std::vector<int64_t> flow_bytes_sys;    // per system and sweep direction: [b * 2 + dir]
  int64_t residual_bytes = 0;          // all colours' local-residual kernels (non-zero e)

  // profiling
  bool profiling = false;
  double prof_ms = 0.0;
  int64_t prof_launches = 0, prof_bytes = 0;
  double prof_idle_ms = 0.0;       // launches that ran for no system (every one had stopped)
  int64_t prof_idle_launches = 0;
  std::vector<hipEvent_t> ev_pool;
  // profiled local-solve launches awaiting their durations: the event pair, the
  // launch (colour c, or 2C + dir for a task-queue sweep direction) and the CG
  // iteration that enqueued it (-1 outside a solve).  Bytes are credited only for
  // the systems that were still iterating when it ran.
  struct PendingLaunch {
    int ev;
    int32_t what;
    int32_t tag;
  };
  std::vector<PendingLaunch> pending;
  int32_t cur_tag = -1;   // CG iteration of the launches being enqueued
  // when set, the next local-solve launch carries this event pair on its own dispatch
  // (start and end of the kernel itself, not markers queued around it)
  mutable hipEvent_t kev0 = nullptr, kev1 = nullptr;
  int ev_used = 0;

  ~Handle();
};

inline Handle* H(ddg_handle p) { return reinterpret_cast<Handle*>(p); }

// Runs fn and turns every exception into a status code and the thread-local message.
template <class Fn>
int guarded(Fn&& fn) {
  try {
    clear_error();
    fn();
    return DDG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return DDG_ERR_OOM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return DDG_ERR_HIP;
  }
}

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip translation units)

// The handle's diagonal storage of A for the row-dot kernels (diag null: CSR rows).
inline DiaView dia_view(const Handle& h) {
  DiaView d{};
  if (h.dia_ok) {
    d.diag = h.dia_diag.as<double>();
    d.up = h.dia_up.as<double>();
    d.sys = h.dia_sys.as<DiaSys>();
  }
  d.n = h.S.n;
  d.nb = h.nb;
  return d;
}
// Refill the diagonals from the CSR values and count entries whose transpose
// differs in its bits (into err_flag[4]).
void launch_dia_refresh(Handle& h, hipStream_t s);

// cg kernels
void launch_fill(double* x, double v, int64_t n, hipStream_t s);
void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);
void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s);
// CG: init (x = 0, r = f, ||f||), then rho = r^T z and p = z, then per iteration
// q = A p / alpha / x,r update / convergence, and after M^{-1}: rho', beta, p = z + beta p.
void launch_cg_init(Handle& h, const double* f, double* x, hipStream_t s);
void launch_cg_start(Handle& h, hipStream_t s);
void launch_cg_step_a(Handle& h, double* x, hipStream_t s);
void launch_cg_step_b(Handle& h, hipStream_t s);
void launch_true_residual(Handle& h, const double* f, const double* x, hipStream_t s);
void build_cg_map(Handle& h, hipStream_t s);

// preconditioner
// guard: CG states whose done flags the kernels obey (default: the handle's own when
// guarded, none otherwise); the coarse level of a three-level handle obeys the fine one's
void launch_precond(Handle& h, const double* r, double* e, int32_t stages, bool guarded,
                    hipStream_t s, const CgState* guard = nullptr);
// one sweep direction (0: colours ascending, 1: descending) as a persistent launch
void launch_sweep_flow(Handle& h, int dir, const double* r, double* e, const CgState* st, hipStream_t s);
void prepare_persist(Handle& h, hipStream_t s);
void prepare_ic(Handle& h, hipStream_t s);
void launch_ic_factor(Handle& h, hipStream_t s);
void launch_ic_solve(Handle& h, const CgState* st, const double* b0, double* y, hipStream_t s);
void launch_persist(Handle& h, const double* f, double* x, hipStream_t s);

// setup numerics
void launch_coarse_basis(Handle& h, hipStream_t s);
void launch_q_own(Handle& h, hipStream_t s);   // Qo and qpos from Q
void launch_galerkin(Handle& h, hipStream_t s);
void launch_coarse_invert(Handle& h, hipStream_t s);
// max over systems of ||v - X A0 v|| / ||v|| for a fixed pseudo-random v (X the packed inverse)
void launch_coarse_measure(Handle& h, hipStream_t s);
double finish_coarse_measure(const Handle& h);
// F0 = R0 F (nc_pad x k column-major, zero padding) from the device copy of F
void launch_restrict_columns(Handle& h, double* F0, hipStream_t s);
void launch_local_factor(Handle& h, hipStream_t s);
void launch_refresh_couplings(Handle& h, hipStream_t s);
// dst[t] = src[pos[t]] (0 where pos[t] < 0), t < m
void launch_gather(const int64_t* pos, const double* src, double* dst, int64_t m, hipStream_t s);

}  // namespace ddg
