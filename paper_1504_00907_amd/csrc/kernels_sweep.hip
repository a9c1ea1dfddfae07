// Colour phase of the multiplicative Schwarz sweep (Section 6 update equation):
// for every subdomain i of one colour, concurrently,
//     e[set_i] += A_i^{-1} (r - A e)[set_i].
// Same-colour subdomains never touch each other's set or its neighbourhood
// (conflict colouring), so the phase is race-free and deterministic.
//
// Local solve.  A_i is block tridiagonal over the K levels of its ascending
// ordering (D_k diagonal blocks, L_k = A_{k,k-1}, U_k = A_{k,k+1}).  The
// factorisation is "twisted": with a middle level m (chosen per subdomain on
// the host so that the two chains carry about the same work) it eliminates levels
// 0..m-1 from the top (X+_k = S+_k^{-1}, S+_k = D_k - L_k X+_{k-1} L_k^T),
// levels K-1..m+1 from the bottom (X-_k, S-_k = D_k - U_k X-_{k+1} U_k^T)
// and stores X_m for the middle level S_m = D_m - L_m X+ L_m^T - U_m X- U_m^T.
// The exact solve of A_i x = b is then
//   forward:  t_k = X+_k (b_k - L_k t_{k-1})   k = 0..m-1
//             t_k = X-_k (b_k - U_k t_{k+1})   k = K-1..m+1
//   middle:   x_m = X_m (b_m - L_m t_{m-1} - U_m t_{m+1})
//   backward: x_k = t_k - X+_k U_k x_{k+1}     k = m-1..0
//             x_k = t_k - X-_k L_k x_{k-1}     k = m+1..K-1
// Each X product is a tiled symmetric GEMV (symv_tile.hpp) that streams the
// factor from HBM once per substitution.  The two chains are independent up to
// the middle level, so a subdomain can be split over two workgroups that hand
// over one level vector each way (t_{m+1} up, x_m down).
//
// Every wave loads all of its tiles of a level at once and, as soon as it has
// used them, issues the loads of the next level, so the HBM latency overlaps
// the reductions and barriers between levels.
#include <cstdlib>

#include <hip/hip_ext.h>

#include "cg_device.hpp"
#include "coarse_device.hpp"
#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

struct SweepArgs {
  const int32_t* subs;
  int32_t nsub;
  int32_t twisted;
  const int64_t* set_ptr;
  const int32_t* set_idx;
  const int32_t* sub_blk_ptr;
  const int32_t* sub_mid;   // middle level of each subdomain's twisted factorisation
  const int32_t* blk_start;
  const int32_t* blk_size;
  const int64_t* blk_foff;
  const int32_t* lo_col;
  const double* lo_val;
  const int32_t* up_col;
  const double* up_val;
  int32_t cl, cu;
  // sliced couplings (rows with more than kCplRegs couplings in a direction)
  const int32_t* blk_slice;
  const int64_t* sl_lo_off;
  const int64_t* sl_up_off;
  const int32_t* sl_lo_col;
  const int32_t* sl_up_col;
  const void* sl_lo_val;   // in the sweep's arithmetic type
  const void* sl_up_val;
  int32_t tab_n;           // entries of each on-chip slice-offset table (most slices of a subdomain + 1)
  int32_t tab_bytes;       // on-chip bytes of both tables (0 without sliced couplings)
  const int64_t* rp;
  const int32_t* ci;
  const double* val;
  int lpr;          // lanes per CSR row of the residual rows (as k_local_residual<L>)
  const void* fac;
  const double* r;
  double* e;
  const double* bres;  // local residuals of this colour's sets, indexed like set_idx
  const CgState* st;         // per system; a subdomain is skipped once its system has stopped
  const int32_t* sub_inst;   // system of each subdomain
  int32_t e_zero;
  int32_t ldp;      // per-wave partial row length (>= max padded block rows)
  double* xch;      // per subdomain: 2 * xch_ld values
  int32_t* flags;   // per subdomain: 2 flags
  int32_t xch_ld;
  int32_t* err;
  int32_t slot_tiles;   // tiles whose partial slots fit on chip (a multiple of one round); wider
                        // levels are reduced in phases of this many tiles into an accumulator
  // grouped launch (several workgroups per chain, wide levels split between them)
  int32_t groups;        // workgroups per chain (1 otherwise)
  int32_t split_rounds;  // a level of at least this many rounds (>= 2) is split over the group
  void* gx;              // per (slot, chain): 2 parities x groups x xch_ld partial level sums
  int32_t* gcnt;         // per (slot, chain): barrier count
  // bounded waits: polls before a wait gives up and raises the error flag, and a
  // test switch that leaves waits unsatisfied (bit 0: the chain handoff is never
  // signalled; bit 1: the first workgroup of a group never counts itself at a barrier)
  int32_t spin_limit;
  int32_t fault;
};

namespace {

enum StepKind { FWD_LO = 0, FWD_UP = 1, MID = 2, BWD_UP = 3, BWD_LO = 4 };

// Step s of a workgroup's sequence.  role 0: whole subdomain; 1: top chain and
// middle; 2: bottom chain.
__device__ inline void decode_step(int role, int s, int K, int m, int& kind, int& k) {
  const int nB = K - 1 - m;
  if (role == 1) {
    if (s < m) { kind = FWD_LO; k = s; }
    else if (s == m) { kind = MID; k = m; }
    else { kind = BWD_UP; k = m - 1 - (s - m - 1); }
    return;
  }
  if (role == 2) {
    if (s < nB) { kind = FWD_UP; k = K - 1 - s; }
    else { kind = BWD_LO; k = m + 1 + (s - nB); }
    return;
  }
  if (s < m) { kind = FWD_LO; k = s; }
  else if (s < m + nB) { kind = FWD_UP; k = K - 1 - (s - m); }
  else if (s == m + nB) { kind = MID; k = m; }
  else if (s < 2 * m + nB + 1) { kind = BWD_UP; k = m - 1 - (s - m - nB - 1); }
  else { kind = BWD_LO; k = m + 1 + (s - 2 * m - nB - 1); }
}

constexpr int kSpinLimit = 1 << 22;

// Explicit vmcnt(0) (expcnt and lgkmcnt left alone).  After an agent-scope release
// it makes the L2 write-back finish before the flag or count that follows: once
// every wave has waited for its own stores before the barrier, the compiler's wait
// pass counts no outstanding vector-memory operation and drops the wait that the
// release fence carries, and the write-back is not counted.  After an agent-scope
// acquire it makes the cache invalidation finish before the barrier lets the other
// waves load.
__device__ inline void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Bounded wait for the partner workgroup's flag.  Only thread 0 polls and
// performs the agent-scope acquire (which invalidates this CU's vector cache and
// the die's L2 lines); the barrier then orders every wave's reads of the exchange
// buffer after it.  The reader clears the flag for the next launch.
__device__ inline void handoff_wait(int32_t* flag, int32_t* err, int sub, int limit) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > limit) {
        if (atomicCAS(err, 0, DDG_ERR_HIP) == 0) {
          err[1] = sub;
          err[2] = -7;
        }
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    wait_vm();
    __hip_atomic_store(flag, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
}

// Publish the exchange buffer: every wave waits for its own stores to
// complete (vmcnt 0), the barrier collects the waves, and thread 0 issues one
// agent-scope release before raising the flag.
// (n flags: one per reading workgroup of a grouped launch)
__device__ inline void handoff_signal(int32_t* flag, int n = 1) {
  wait_vm();
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    wait_vm();
    for (int i = 0; i < n; ++i) __hip_atomic_store(flag + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Barrier of the workgroups of one chain in a grouped launch: every wave waits for
// its own stores, thread 0 makes an agent-scope release, counts the workgroup and
// waits (bounded; also ended by an error another workgroup raised) until the count
// reaches `target`, then makes an agent-scope acquire before the barrier lets the
// other waves read.
__device__ inline void group_barrier(int32_t* cnt, int target, int32_t* err, int sub, int limit, bool count) {
  wait_vm();
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    wait_vm();
    if (count) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (spins > limit) {
        if (atomicCAS(err, 0, DDG_ERR_HIP) == 0) {
          err[1] = sub;
          err[2] = -11;
        }
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    wait_vm();
  }
  __syncthreads();
}

}  // namespace

// c + sum_{q >= q0} val_q * w[col_q] over the entries of one row of a slice (lane
// ln), in the order the entries are stored; the slice's entries are
// [base + tab[sl], base + tab[sl + 1]), 64 per entry index.  The slice's width is
// the same for all lanes of a wave, so the loads are coalesced; they go out in
// chunks of cpl_chunk<AT>() entries, the next chunk's before the current one is
// used (two chunks in flight, one dependent round trip per chunk pair rather than
// per chunk), and the last chunk is predicated rather than taken one entry at a
// time.  (FP64 values take half-size chunks: the same registers as one FP32 chunk pair.)
template <class AT>
__host__ __device__ constexpr int cpl_chunk() { return sizeof(AT) == 8 ? 4 : 8; }
// entries of the first row a thread owns in a level, prefetched one level ahead
constexpr int kCplHead = 4;

template <class AT>
__device__ inline AT slice_dot(const int32_t* tab, int64_t base, const int32_t* __restrict__ col,
                               const AT* __restrict__ val, int sl, int ln, int q0, const AT* w, AT c) {
  constexpr int U = cpl_chunk<AT>();
  const int n = ((tab[sl + 1] - tab[sl]) >> 6) - q0;   // entries left in the row
  const int64_t o0 = base + tab[sl] + 64 * q0 + ln;
  int cc[U], cn[U];
  AT vv[U], vn[U];
  auto load = [&](int i, int (&cx)[U], AT (&vx)[U]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = i * U + u;
      cx[u] = 0;
      vx[u] = 0;
      if (q < n) {
        cx[u] = col[o0 + 64 * q];
        vx[u] = val[o0 + 64 * q];
      }
    }
  };
  if (n > 0) load(0, cc, vv);
  for (int i = 0; i * U < n; ++i) {
    if ((i + 1) * U < n) load(i + 1, cn, vn);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i * U + u < n) c += vv[u] * w[cc[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cc[u] = cn[u];
      vv[u] = vn[u];
    }
  }
  return c;
}

constexpr int kMaxLevels = 96;   // levels per subdomain staged in LDS

// One local solve: subdomain `sub`, chain `role` (0: whole subdomain; 1: top chain
// and middle level; 2: bottom chain), exchange slot `xs` of the two-workgroup
// handoff.  SL = false: at most kCplRegs couplings per row and direction (held in
// registers, rows past the first NT of a level read the ELL arrays); SL = true:
// the sliced coupling layout.  OWN_RES: the workgroup forms b = (r - A e) on its
// own rows from the CSR rows of A (res_e_zero: e is zero there) instead of reading
// the local-residual kernel's output.  GRP: workgroup gi of the a.groups that share
// the chain; a level of at least a.split_rounds rounds is split between them (each
// sums the slots of its own rounds, the partial sums are exchanged through global
// memory and added in workgroup order, so all of them hold the same level result);
// a narrower level is computed whole by each of them.
template <class FT, class AT, int T, int NW, int TPW, bool SL, bool OWN_RES, bool GRP = false>
__device__ inline void sweep_task(const SweepArgs& a, int sub, int role, int xs, bool res_e_zero, int gi = 0) {
  using G = TileGeom<FT, T>;
  constexpr int NT = NW * 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int32_t lv_start[kMaxLevels + 1], lv_size[kMaxLevels];
  __shared__ int64_t lv_foff[kMaxLevels];
  __shared__ int32_t lv_slice[kMaxLevels];  // first slice of each level, relative to the subdomain's
  const int p = xs;
  constexpr int NWT = NW * TPW;
  const int NG = GRP ? a.groups : 1;   // workgroups of the chain
  // this workgroup's rounds [rf, rl) of a level of ntl_ tiles (empty for some
  // workgroups when a split level has fewer rounds than the group has workgroups)
  auto rounds_of = [&](int ntl_, int& rf, int& rl) __attribute__((always_inline)) {
    const int R = (ntl_ + NWT - 1) / NWT;
    rf = 0;
    rl = R;
    if constexpr (GRP) {
      if (R >= a.split_rounds) {
        rf = R * gi / NG;
        rl = R * (gi + 1) / NG;
      }
    }
  };
  const int64_t s0 = a.set_ptr[sub];
  const int ni = (int)(a.set_ptr[sub + 1] - s0);
  const int ni_pad = (ni + 3) & ~3;
  // sliced couplings: per-slice entry offsets of this subdomain, relative to its first entry
  int32_t* tab_lo = reinterpret_cast<int32_t*>(smem_raw);
  int32_t* tab_up = tab_lo + a.tab_n;
  AT* w = reinterpret_cast<AT*>(smem_raw + a.tab_bytes);
  AT* tv = w + ni_pad;
  AT* acc = tv + a.ldp;     // phase accumulator (levels wider than slot_tiles only)
  AT* slots = acc + a.ldp;  // 2 * T per tile of the current phase
  // the wave index is read as wave-uniform where the tile loads find kept lanes
  // (edges 32 and 64: it keeps their index arithmetic scalar); at edge 16 the plain
  // index compiles to the faster kernel
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = short_last_row(T) ? __builtin_amdgcn_readfirstlane(tid >> 6) : (tid >> 6);
  const FT* fac = static_cast<const FT*>(a.fac);
  const int kb0 = a.sub_blk_ptr[sub];
  const int K = a.sub_blk_ptr[sub + 1] - kb0;  // <= kMaxLevels (checked on the host)
  for (int k = tid; k < K; k += NT) {
    lv_start[k] = a.blk_start[kb0 + k];
    lv_size[k] = a.blk_size[kb0 + k];
    lv_foff[k] = a.blk_foff[kb0 + k];
  }
  int64_t base_lo = 0, base_up = 0;
  if constexpr (SL) {
    const int sl0 = a.blk_slice[kb0];
    const int nsl = a.blk_slice[kb0 + K] - sl0;  // < tab_n (checked on the host)
    base_lo = a.sl_lo_off[sl0];
    base_up = a.sl_up_off[sl0];
    for (int k = tid; k < K; k += NT) lv_slice[k] = a.blk_slice[kb0 + k] - sl0;
    for (int t = tid; t <= nsl; t += NT) {
      tab_lo[t] = (int32_t)(a.sl_lo_off[sl0 + t] - base_lo);
      tab_up[t] = (int32_t)(a.sl_up_off[sl0 + t] - base_up);
    }
  }
  const int m = a.sub_mid[sub];
  const int nB = K - 1 - m;
  const int split = (m + 1 < K) ? a.blk_start[kb0 + m + 1] : ni;  // first row of the bottom chain
  int r0 = 0, r1 = ni;
  if (role == 1) r1 = split;
  if (role == 2) r0 = split;
  const int ns = role == 0 ? 2 * K - 1 : (role == 1 ? 2 * m + 1 : 2 * nB);

  __syncthreads();  // level metadata visible

  FT R[TPW][G::SS];
  // the wave's first-round tiles are the same at every level
  int tI[TPW], tJ[TPW];
#pragma unroll
  for (int j = 0; j < TPW; ++j) tile_ij(j * NW + wave, tI[j], tJ[j]);
  // tile t = (I, J) of level k into register set j
  constexpr bool CD = compact_diag(T);
  // this lane's place in a compact diagonal tile (p >= q lanes kept)
  const bool dkept = lane_p(lane) >= lane_q(lane);
  const int dslot = __builtin_popcountll(kept_lanes(8, true, true) & ((1ull << lane) - 1ull));
  const unsigned long long below = (1ull << lane) - 1ull;
  auto load_tile_at = [&](int k, int t, int I, int J, int j) __attribute__((always_inline)) {
    if constexpr (!short_last_row(T) && !CD) {
      // full tiles only
      load_subtile<FT, T>(fac + lv_foff[k] + (int64_t)t * T * T, lane, R[j]);
      return;
    }
    const int bk = __builtin_amdgcn_readfirstlane(lv_size[k]);
    const int ntk = (bk + T - 1) / T;
    bool kept = true;
    int c = lane, nk = 64, ph = 8;
    if (I == ntk - 1) {
      // short last tile-row: the kept lanes of its tiles (wave-uniform mask)
      ph = last_row_subtiles(bk, T);
      const unsigned long long mask = kept_lanes_rt<CD>(ph, I == J);
      kept = (mask >> lane) & 1ull;
      c = __builtin_popcountll(mask & below);
      nk = __builtin_popcountll(mask);
    } else if (CD && I == J) {
      kept = dkept;
      c = dslot;
      nk = kDiagLanes;
    }
    const FT* src = fac + lv_foff[k] + tile_off<FT, T>(t, I, J, ntk, ph);
    if (nk == 64) load_subtile<FT, T>(src, lane, R[j]);  // full tile: constant chunk offsets
    else load_subtile_at<FT, T>(src, kept, c, nk, R[j]);
  };
  // coupling entries of this thread's row (row tid of the level) for the next step
  int cpl_col[2 * kCplRegs];
  AT cpl_val[2 * kCplRegs];
  constexpr bool cpl_regs = !SL;
  auto load_tile = [&](int k, int j) __attribute__((always_inline)) {
    const int ntl = tiles_for(lv_size[k], T);
    if constexpr (GRP) {
      // this workgroup's first tile of slot j at level k
      int rf, rl;
      rounds_of(ntl, rf, rl);
      const int t = (rf * TPW + j) * NW + wave;
      if (rf < rl && t < ntl) {
        int I = tI[j], J = tJ[j];
        if (rf > 0) tile_ij(t, I, J);
        load_tile_at(k, t, I, J, j);
      }
    } else {
      const int t = j * NW + wave;
      if (t < ntl) load_tile_at(k, t, tI[j], tJ[j], j);
    }
  };
  auto load_cpl = [&](int kind, int k) {
    if (!cpl_regs) return;
    const int b = lv_size[k];
    const bool use_lo = (kind == FWD_LO || kind == MID || kind == BWD_LO);
    const bool use_up = (kind == FWD_UP || kind == MID || kind == BWD_UP);
    const int64_t row = s0 + lv_start[k] + tid;
#pragma unroll
    for (int q = 0; q < kCplRegs; ++q) {
      cpl_col[q] = -1;
      cpl_col[kCplRegs + q] = -1;
      cpl_val[q] = 0;
      cpl_val[kCplRegs + q] = 0;
      if (tid < b) {
        if (use_lo && q < a.cl) {
          cpl_col[q] = a.lo_col[row * a.cl + q];
          cpl_val[q] = (AT)a.lo_val[row * a.cl + q];
        }
        if (use_up && q < a.cu) {
          cpl_col[kCplRegs + q] = a.up_col[row * a.cu + q];
          cpl_val[kCplRegs + q] = (AT)a.up_val[row * a.cu + q];
        }
      }
    }
  };
  // sliced couplings: the first kCplHead entries of row tid of the next step's level,
  // per direction (hw = the slice's width, 0 when the direction is unused)
  int hcol[2][kCplHead];
  AT hval[2][kCplHead];
  int hw[2] = {0, 0};
  auto load_head = [&](int kind, int k) {
    if constexpr (SL) {
      const int b = lv_size[k];
      const bool use[2] = {kind == FWD_LO || kind == MID || kind == BWD_LO,
                           kind == FWD_UP || kind == MID || kind == BWD_UP};
      const int slr = lv_slice[k] + wave;  // slice of row tid (valid when tid < b)
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        hw[d] = 0;
        if (use[d] && tid < b) {
          const int32_t* tab = d ? tab_up : tab_lo;
          const int64_t o = (d ? base_up : base_lo) + tab[slr] + lane;
          hw[d] = (tab[slr + 1] - tab[slr]) >> 6;
          const int32_t* col = d ? a.sl_up_col : a.sl_lo_col;
          const AT* val = static_cast<const AT*>(d ? a.sl_up_val : a.sl_lo_val);
#pragma unroll
          for (int u = 0; u < kCplHead; ++u)
            if (u < hw[d]) {
              hcol[d][u] = col[o + 64 * u];
              hval[d][u] = val[o + 64 * u];
            }
        }
      }
    }
  };
  // 1. local residual b = (r - A e) on the rows this workgroup owns; with sliced
  //    couplings the other chain's rows start at zero (the handoff writes the ones
  //    that are read).  OWN_RES: formed here from the CSR rows of A before the first
  //    level's tiles are requested (its loads then hold no tile registers); otherwise
  //    the first level's couplings and tiles are requested first and the residual
  //    that k_local_residual wrote is read after them (vector loads complete in
  //    issue order, so a wait for the couplings does not wait for the tiles).
  auto prefetch_first = [&]() {
    if (ns > 0) {
      int kind, k;
      decode_step(role, 0, K, m, kind, k);
      load_cpl(kind, k);
      load_head(kind, k);
#pragma unroll
      for (int j = 0; j < TPW; ++j) load_tile(k, j);
    }
  };
  if constexpr (SL) {
    for (int j = tid; j < ni; j += NT)
      if (j < r0 || j >= r1) w[j] = (AT)0;
  }
  if constexpr (OWN_RES) {
    // the same arithmetic as k_local_residual<lpr>, so both schedules agree bit for bit
    const int L = a.lpr;
    if (L == 1) {
      for (int j = r0 + tid; j < r1; j += NT) {
        const int g = a.set_idx[s0 + j];
        const double rg = a.r[g];
        w[j] = (AT)(res_e_zero ? rg : row_sub(a.rp, a.ci, a.val, a.e, g, rg));
      }
    } else {
      const int lg = tid & (L - 1);
      for (int j = r0 + tid / L; j < r1; j += NT / L) {  // a lane group shares j
        const int g = a.set_idx[s0 + j];
        const double ae = res_e_zero ? 0.0 : row_dot_rt(a.rp, a.ci, a.val, a.e, g, lg, L);
        if (lg == 0) w[j] = (AT)(a.r[g] - ae);
      }
    }
    prefetch_first();
  } else {
    prefetch_first();
    for (int j = r0 + tid; j < r1; j += NT) w[j] = (AT)a.bres[s0 + j];
  }
  __syncthreads();

  double* xch = a.xch + (int64_t)p * 2 * a.xch_ld;
  // handoff flags of the slot: [d * NG + i] for direction d (0: up to the top chain,
  // 1: down to the bottom chain) and reading workgroup i
  int32_t* flags = a.flags + 2 * p * NG;
  // grouped launch: this chain's partial-sum buffers and barrier count, and the
  // number of split levels passed so far
  const int chain = 2 * p + (role == 2 ? 1 : 0);
  int32_t* gcnt = GRP ? a.gcnt + chain : nullptr;
  int nsplit = 0;

  for (int s = 0; s < ns; ++s) {
    int kind, k;
    decode_step(role, s, K, m, kind, k);
    const int bs = lv_start[k];
    const int b = lv_size[k];
    const int nt = (b + T - 1) / T;
    const int ntl = nt * (nt + 1) / 2;
    if (role == 1 && kind == MID && nB > 0) {
      // import t_{m+1} from the bottom chain
      handoff_wait(flags + gi, a.err, sub, a.spin_limit);
      const int bs1 = lv_start[m + 1], b1 = lv_size[m + 1];
      for (int jj = tid; jj < b1; jj += NT) w[bs1 + jj] = (AT)xch[jj];
      __syncthreads();
    }
    if (role == 2 && kind == BWD_LO && k == m + 1) {
      // import x_m from the top chain
      handoff_wait(flags + NG + gi, a.err, sub, a.spin_limit);
      const int bsm = lv_start[m], bm = lv_size[m];
      for (int jj = tid; jj < bm; jj += NT) w[bsm + jj] = (AT)xch[a.xch_ld + jj];
      __syncthreads();
    }
    // input vector of this level
    const bool fwd = kind <= MID;
    const bool use_lo = (kind == FWD_LO || kind == MID || kind == BWD_LO);
    const bool use_up = (kind == FWD_UP || kind == MID || kind == BWD_UP);
    for (int jj = tid; jj < nt * T; jj += NT) {
      AT y = 0;
      if (jj < b) {
        AT c = 0;
        if constexpr (SL) {
          const int slr = lv_slice[k] + (jj >> 6);
          const bool use[2] = {use_lo, use_up};
#pragma unroll
          for (int d = 0; d < 2; ++d) {
            if (!use[d]) continue;
            int q0 = 0;
            if (jj == tid) {
              // prefetched head
#pragma unroll
              for (int u = 0; u < kCplHead; ++u)
                if (u < hw[d]) c += hval[d][u] * w[hcol[d][u]];
              q0 = kCplHead;
            }
            c = slice_dot<AT>(d ? tab_up : tab_lo, d ? base_up : base_lo, d ? a.sl_up_col : a.sl_lo_col,
                              static_cast<const AT*>(d ? a.sl_up_val : a.sl_lo_val), slr, jj & 63, q0, w, c);
          }
        } else if (jj == tid) {
#pragma unroll
          for (int q = 0; q < 2 * kCplRegs; ++q)
            if (cpl_col[q] >= 0) c += cpl_val[q] * w[cpl_col[q]];
        } else {
          // rows past the first NT of a wide level: at most kCplRegs couplings each
          const int64_t row = s0 + bs + jj;
          if (use_lo)
            for (int q = 0; q < a.cl; ++q) {
              const int col = a.lo_col[row * a.cl + q];
              if (col >= 0) c += (AT)a.lo_val[row * a.cl + q] * w[col];
            }
          if (use_up)
            for (int q = 0; q < a.cu; ++q) {
              const int col = a.up_col[row * a.cu + q];
              if (col >= 0) c += (AT)a.up_val[row * a.cu + q] * w[col];
            }
        }
        y = fwd ? w[bs + jj] - c : c;
      }
      tv[jj] = y;
    }
    __syncthreads();
    // tiles: the first TPW*NW are already in registers; every wave runs all of its
    // slots (invalid ones on stale registers, without storing) so the tile
    // computations can interleave.  When a level fits in one round, each register
    // set is refilled with the next level's tile as soon as it has been used.
    const int rounds = (ntl + NW * TPW - 1) / (NW * TPW);
    int rf = 0, rl = rounds;   // this workgroup's rounds
    if constexpr (GRP) rounds_of(ntl, rf, rl);
    const bool split = GRP && rounds >= a.split_rounds;
    const int phase_rounds = a.slot_tiles / (NW * TPW);
    const bool phased = split || ntl > a.slot_tiles;
    int kind2 = 0, k2 = 0;
    const bool has_next = s + 1 < ns;
    if (has_next) decode_step(role, s + 1, K, m, kind2, k2);
    for (int round = rf; round < rl; ++round) {
      const int t_phase = GRP ? (rf + ((round - rf) / phase_rounds) * phase_rounds) * NW * TPW
                              : (round / phase_rounds) * phase_rounds * NW * TPW;  // first tile of the phase
      int rI[TPW], rJ[TPW];
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        rI[j] = tI[j];
        rJ[j] = tJ[j];
        if (round > 0) tile_ij((round * TPW + j) * NW + wave, rI[j], rJ[j]);
      }
      if (round > rf) {
#pragma unroll
        for (int j = 0; j < TPW; ++j) {
          const int t = (round * TPW + j) * NW + wave;
          if (t < ntl) load_tile_at(k, t, rI[j], rJ[j], j);
        }
      }
      const bool last = round + 1 == rl;
      if (last && has_next) {
        // the next step's couplings go out before its tiles
        load_cpl(kind2, k2);
        load_head(kind2, k2);
      }
#pragma unroll
      for (int j = 0; j < TPW; ++j) {
        const int t = (round * TPW + j) * NW + wave;
        const bool valid = t < ntl;
        const int I = valid ? rI[j] : 0, J = valid ? rJ[j] : 0;
        symv_tile_slots<FT, AT, T, CD>(R[j], I, J, tv, slots + (int64_t)(2 * (t - t_phase)) * T,
                                       slots + (int64_t)(2 * (t - t_phase) + 1) * T, lane, valid);
        if (last && has_next) load_tile(k2, j);
      }
      if (phased && ((round + 1 - rf) % phase_rounds == 0 || last)) {
        // fold this phase's slots into the accumulator, rows in a fixed tile order
        __syncthreads();
        const int t_end = min(GRP ? min(ntl, rl * NW * TPW) : ntl, t_phase + phase_rounds * NW * TPW);
        for (int jj = tid; jj < b; jj += NT) {
          const AT part = sum_slots_range<AT, T, CD>(slots, nt, jj, t_phase, t_end);
          acc[jj] = t_phase == rf * NW * TPW ? part : acc[jj] + part;
        }
        __syncthreads();
      }
    }
    if (GRP && rl == rf && has_next) {
      // no round of this level here: the next step's couplings and tiles go out now
      load_cpl(kind2, k2);
      load_head(kind2, k2);
#pragma unroll
      for (int j = 0; j < TPW; ++j) load_tile(k2, j);
    }
    __syncthreads();
    if (split) {
      // the group's partial sums of this level (parity of the split count: a buffer
      // is written again only after every workgroup has passed the next barrier,
      // i.e. has read it), summed in workgroup order
      AT* X = static_cast<AT*>(a.gx) + ((int64_t)chain * 2 + (nsplit & 1)) * NG * a.xch_ld;
      for (int jj = tid; jj < b; jj += NT) X[(int64_t)gi * a.xch_ld + jj] = rl > rf ? acc[jj] : (AT)0;
      ++nsplit;
      group_barrier(gcnt, NG * nsplit, a.err, sub, a.spin_limit, !((a.fault & 2) && gi == 0));
      for (int jj = tid; jj < b; jj += NT) {
        AT sum = X[jj];
        for (int i = 1; i < NG; ++i) sum += X[(int64_t)i * a.xch_ld + jj];
        if (fwd) w[bs + jj] = sum;
        else w[bs + jj] -= sum;
      }
    } else {
      for (int jj = tid; jj < b; jj += NT) {
        const AT sum = phased ? acc[jj] : sum_slots<AT, T, CD>(slots, nt, jj);
        if (fwd) w[bs + jj] = sum;
        else w[bs + jj] -= sum;
      }
    }
    __syncthreads();
    // (in a grouped launch every workgroup of a chain holds the same values; the
    // first one hands them over to every workgroup of the other chain)
    if (role == 2 && kind == FWD_UP && k == m + 1 && gi == 0) {
      for (int jj = tid; jj < b; jj += NT) xch[jj] = (double)w[bs + jj];
      if (!(a.fault & 1)) handoff_signal(flags + 0, NG);
    }
    if (role == 1 && kind == MID && nB > 0 && gi == 0) {
      for (int jj = tid; jj < b; jj += NT) xch[a.xch_ld + jj] = (double)w[bs + jj];
      if (!(a.fault & 1)) handoff_signal(flags + NG, NG);
    }
  }

  // scatter-add the correction on the owned rows (in a grouped launch, every G-th
  // block of NT rows by each workgroup)
  constexpr int GB = 4;
  const int gstride = GRP ? NG * NT : NT;
  for (int j0 = r0 + (GRP ? gi * NT : 0) + tid; j0 < r1; j0 += gstride * GB) {
    int g[GB];
    double ev[GB];
#pragma unroll
    for (int q = 0; q < GB; ++q) {
      const int j = j0 + q * gstride;
      g[q] = j < r1 ? a.set_idx[s0 + j] : -1;
    }
#pragma unroll
    for (int q = 0; q < GB; ++q) ev[q] = g[q] >= 0 ? a.e[g[q]] : 0.0;
#pragma unroll
    for (int q = 0; q < GB; ++q)
      if (g[q] >= 0) a.e[g[q]] = ev[q] + (double)w[j0 + q * gstride];
  }
  if constexpr (GRP) {
    // the last workgroup of the chain to get here returns the count to zero for the
    // next launch (every other one has passed all of its waits)
    if (tid == 0 &&
        __hip_atomic_fetch_add(gcnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == NG * (nsplit + 1) - 1)
      __hip_atomic_store(gcnt, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One colour phase: workgroup per (subdomain, chain) of the colour; GRP: a.groups
// workgroups per chain, member i at i times the ungrouped grid (the same XCD when
// the chains are twisted).
template <class FT, class AT, int T, int NW, int TPW, bool SL, bool GRP = false>
__global__ void __launch_bounds__(NW * 64) k_sweep(SweepArgs a) {
  int p, role, gi = 0;
  if constexpr (GRP) {
    const int per = a.twisted ? 16 * ((a.nsub + 7) / 8) : a.nsub;
    gi = blockIdx.x / per;
    const int bx = blockIdx.x - gi * per;
    if (a.twisted) {
      const int g = bx >> 4, w16 = bx & 15;
      p = g * 8 + (w16 & 7);
      role = (w16 < 8) ? 2 : 1;
    } else {
      p = bx;
      role = 0;
    }
  } else if (a.twisted) {
    // pair (bottom, top) = (16g + i, 16g + i + 8): same XCD under round-robin dispatch,
    // bottom chain dispatched first
    const int g = blockIdx.x >> 4, w16 = blockIdx.x & 15;
    p = g * 8 + (w16 & 7);
    role = (w16 < 8) ? 2 : 1;
  } else {
    p = blockIdx.x;
    role = 0;
  }
  if (p >= a.nsub) return;
  const int sub = a.subs[p];
  // both workgroups of a pair read the same flag (stable during the launch), so
  // they skip together and no handoff is left waiting
  if (a.st && a.st[a.sub_inst[sub]].done) return;
  sweep_task<FT, AT, T, NW, TPW, SL, false, GRP>(a, sub, role, p, false, gi);
}

// A whole sweep direction (every colour) as one launch over a task queue.  Tasks
// are (subdomain, chain) in sweep order, colour by colour (bottom chain first).
// Each workgroup, when it starts, takes the next task from a 64-bit counter, waits
// until every earlier subdomain of the sweep that conflicts with its subdomain
// (whose set meets its set's neighbourhood) has finished, forms its residual rows
// and solves.  Subdomains of one colour never conflict, so the corrections and
// every value computed are those of the colour-by-colour launches.  Tasks are
// taken in the order workgroups start, and a task waits only for earlier tasks,
// held by workgroups that are running; a chain's partner is the next task, and
// the workgroups holding earlier tasks never wait for it, so they finish and
// free a slot for it.  Each finished task adds 1 to its subdomain's completion
// count; a dependency is met when the count reaches `target` (chains per
// subdomain times the sweeps launched so far).
struct FlowArgs {
  const int32_t* order;     // subdomains in sweep order
  const int32_t* dep_ptr;   // per subdomain: earlier conflicting subdomains of this sweep
  const int32_t* dep_idx;
  int32_t* done;            // per subdomain completion count
  unsigned long long* counter;
  int64_t base;             // counter value at the start of this launch
  int64_t ntasks;
  int64_t zero_tasks;       // the first zero_tasks tasks start from e = 0
  int32_t roles;            // chains per subdomain (2 with the two-workgroup schedule)
  int32_t target;
};

// Bounded wait for a completion count; gives up at once when an error is already
// flagged, so a failed sweep drains instead of running every wait to its limit.
__device__ inline void flow_wait(const int32_t* cnt, int32_t target, int32_t* err, int sub) {
  int spins = 0;
  while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(2);
    ++spins;
    if ((spins & 255) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
    if (spins > kSpinLimit) {
      if (atomicCAS(err, 0, DDG_ERR_HIP) == 0) {
        err[1] = sub;
        err[2] = -8;
      }
      break;
    }
  }
}

// Wait for every dependency of subdomain `sub`, then acquire.  Kept out of line:
// inlined, its polling loop raises the register allocation of the whole kernel.
__device__ __attribute__((noinline)) void flow_wait_deps(const int32_t* dep_ptr, const int32_t* dep_idx,
                                                         const int32_t* done, int32_t target, int32_t* err,
                                                         int sub) {
  for (int d = dep_ptr[sub]; d < dep_ptr[sub + 1]; ++d) flow_wait(done + dep_idx[d], target, err, sub);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  wait_vm();
}

template <class FT, class AT, int T, int NW, int TPW, bool SL>
__global__ void __launch_bounds__(NW * 64) k_sweep_flow(SweepArgs a, FlowArgs f) {
  __shared__ int64_t task_s;
  if (threadIdx.x == 0) task_s = (int64_t)atomicAdd(f.counter, 1ull) - f.base;
  __syncthreads();
  const int64_t t = task_s;  // in [0, ntasks): one workgroup per task, counter base kept by the host
  if (t < 0 || t >= f.ntasks) {
    if (threadIdx.x == 0 && atomicCAS(a.err, 0, DDG_ERR_HIP) == 0) {
      a.err[1] = -1;
      a.err[2] = -9;
    }
    return;
  }
  const int sub = f.order[t / f.roles];
  const int role = f.roles == 2 ? ((t & 1) ? 1 : 2) : 0;
  if (threadIdx.x == 0) {
    flow_wait_deps(f.dep_ptr, f.dep_idx, f.done, f.target, a.err, sub);
  }
  __syncthreads();
  if (!(a.st && a.st[a.sub_inst[sub]].done))
    sweep_task<FT, AT, T, NW, TPW, SL, true>(a, sub, role, sub, t < f.zero_tasks);
  // publish this chain's corrections of e, then count the task as finished
  wait_vm();
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    wait_vm();
    __hip_atomic_fetch_add(f.done + sub, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// b = (r - A e) on the expanded sets of one colour, written in set order; L lanes
// per CSR row (one row per lane when L = 1, from the diagonals when the handle
// stores them).
template <int L>
__global__ void __launch_bounds__(256) k_local_residual(const CgState* st, const int32_t* __restrict__ sub_inst,
                                                        const int32_t* __restrict__ subs,
                                                        const int64_t* __restrict__ set_ptr,
                                                        const int32_t* __restrict__ set_idx,
                                                        const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                                        const double* __restrict__ val, DiaView D,
                                                        const double* __restrict__ r,
                                                        const double* __restrict__ e, int e_zero,
                                                        double* __restrict__ bres) {
  const int sub = subs[blockIdx.y];
  if (st && st[sub_inst[sub]].done) return;
  const int64_t s0 = set_ptr[sub];
  const int ni = (int)(set_ptr[sub + 1] - s0);
  const int j = blockIdx.x * (256 / L) + threadIdx.x / L;
  if (j >= ni) return;  // the whole lane group leaves together
  const int g = set_idx[s0 + j];
  if constexpr (L == 1) {
    const double rg = r[g];
    if (e_zero) bres[s0 + j] = rg;
    else if (D.diag) bres[s0 + j] = dia_row_sub(D, D.sys[sub_inst[sub]], e, g, rg);
    else bres[s0 + j] = row_sub(rp, ci, val, e, g, rg);
  } else {
    const double ae = e_zero ? 0.0 : row_dot_l<L>(rp, ci, val, e, g, threadIdx.x & (L - 1));
    if ((threadIdx.x & (L - 1)) == 0) bres[s0 + j] = r[g] - ae;
  }
}

namespace {

// flow_dir < 0: one colour phase (its local-residual kernel when `residual`, else its
// local solves); flow_dir = 0 / 1: the whole ascending / descending sweep as one
// persistent launch.
// The local-solve arguments of one launch and its dynamic LDS size (on-chip plan:
// w (set), tv and the phase accumulator (one level each), then the per-tile slots
// of up to slot_tiles tiles, whole rounds of NW * TPW tiles).
template <class FT, class AT, int T, int NW, int TPW, bool SL>
size_t build_sweep_args(const Handle& h, const int32_t* subs, int nsub, const double* r, double* e, bool e_zero,
                        const CgState* st, SweepArgs& a) {
  const Symbolic& S = h.S;
  a.subs = subs;
  a.nsub = nsub;
  a.twisted = h.twisted_ok ? 1 : 0;
  a.set_ptr = h.set_ptr.as<int64_t>();
  a.set_idx = h.set_idx.as<int32_t>();
  a.sub_blk_ptr = h.sub_blk_ptr.as<int32_t>();
  a.sub_mid = h.sub_mid.as<int32_t>();
  a.blk_start = h.blk_start.as<int32_t>();
  a.blk_size = h.blk_size.as<int32_t>();
  a.blk_foff = h.blk_foff.as<int64_t>();
  a.lo_col = h.lo_col.as<int32_t>();
  a.lo_val = h.lo_val.as<double>();
  a.up_col = h.up_col.as<int32_t>();
  a.up_val = h.up_val.as<double>();
  a.cl = S.cl;
  a.cu = S.cu;
  a.blk_slice = h.blk_slice.as<int32_t>();
  a.sl_lo_off = h.sl_lo_off.as<int64_t>();
  a.sl_up_off = h.sl_up_off.as<int64_t>();
  a.sl_lo_col = h.sl_lo_col.as<int32_t>();
  a.sl_up_col = h.sl_up_col.as<int32_t>();
  a.sl_lo_val = h.sl_lo_val.p;
  a.sl_up_val = h.sl_up_val.p;
  DDG_REQUIRE(S.sliced == !(S.cl <= kCplRegs && S.cu <= kCplRegs), DDG_ERR_HIP, "internal: coupling layout");
  a.lpr = h.lpr;
  a.rp = h.rowptr.as<int64_t>();
  a.ci = h.col.as<int32_t>();
  a.val = h.val.as<double>();
  a.fac = h.fac.p;
  a.r = r;
  a.e = e;
  a.bres = h.ws.bres;
  a.st = st;
  a.sub_inst = h.sub_inst.as<int32_t>();
  a.e_zero = e_zero ? 1 : 0;
  const int maxpad = ((S.max_blk + T - 1) / T) * T;
  a.ldp = maxpad;
  a.xch = h.xch.as<double>();
  a.flags = h.flags.as<int32_t>();
  a.xch_ld = h.xch_ld;
  a.err = h.err_flag.as<int32_t>();
  a.groups = 1;
  a.split_rounds = 1 << 30;
  // DDG_SPIN_LIMIT / DDG_SWEEP_FAULT: shorter bounded waits and unsatisfied waits for
  // the tests of the error paths (read at every launch, so a test can clear them)
  a.spin_limit = kSpinLimit;
  if (const char* env = std::getenv("DDG_SPIN_LIMIT")) a.spin_limit = std::max(16, std::atoi(env));
  a.fault = 0;
  if (const char* env = std::getenv("DDG_SWEEP_FAULT")) a.fault = std::atoi(env);
  a.gx = h.gx.p;
  a.gcnt = h.gcnt.as<int32_t>();
  const int ni_pad = (S.max_set + 3) & ~3;
  DDG_REQUIRE(S.max_blocks <= kMaxLevels, DDG_ERR_UNSUPPORTED, "more than 96 levels in a local problem");
  const int max_tiles = tiles_for(S.max_blk, T);
  // on-chip plan: w (set), tv and the phase accumulator (one level each), then the
  // per-tile slots of up to slot_tiles tiles (whole rounds of NW * TPW tiles)
  const int round_tiles = NW * TPW;
  a.tab_n = SL ? S.max_sub_slices + 1 : 0;
  a.tab_bytes = (int32_t)(((int64_t)2 * a.tab_n * 4 + 15) / 16 * 16);
  const int64_t fixed = a.tab_bytes + sizeof(AT) * ((int64_t)ni_pad + 2 * (int64_t)maxpad);
  const int64_t per_tile = sizeof(AT) * 2 * (int64_t)T;
  // (the kernel's static level metadata takes about 1.9 KiB of the same LDS)
  int64_t cap = (h.dev_lds_limit - 2048 - fixed) / per_tile;
  cap = cap / round_tiles * round_tiles;
  if (const char* env = std::getenv("DDG_SWEEP_SLOT_TILES")) cap = std::min<int64_t>(cap, std::max(1, std::atoi(env)) * (int64_t)round_tiles);
  const int64_t need_tiles = (int64_t)(max_tiles + round_tiles - 1) / round_tiles * round_tiles;
  a.slot_tiles = (int32_t)std::min<int64_t>(cap, need_tiles);
  DDG_REQUIRE(a.slot_tiles >= round_tiles, DDG_ERR_UNSUPPORTED,
              "local problem too large for on-chip storage (" + std::to_string(fixed) + " bytes before slots)");
  return (size_t)(fixed + per_tile * a.slot_tiles);
}

template <class FT, class AT, int T, int NW, int TPW, bool SL>
void launch_sweep_cfg(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                      const CgState* st, hipStream_t s, bool residual, int flow_dir) {
  const Symbolic& S = h.S;
  const int nsub = flow_dir >= 0 ? S.n_parts : S.colour_ptr[colour + 1] - S.colour_ptr[colour];
  if (nsub == 0) return;
  SweepArgs a;
  const size_t lds = build_sweep_args<FT, AT, T, NW, TPW, SL>(
      h, h.colour_subs.as<int32_t>() + (flow_dir >= 0 ? 0 : S.colour_ptr[colour]), nsub, r, e, e_zero, st, a);
  if (flow_dir >= 0) {
    auto fk = k_sweep_flow<FT, AT, T, NW, TPW, SL>;
    if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    FlowArgs f;
    f.roles = h.twisted_ok ? 2 : 1;
    f.ntasks = (int64_t)f.roles * S.n_parts;
    f.zero_tasks = flow_dir == 0 && e_zero ? (int64_t)f.roles * (S.colour_ptr[1] - S.colour_ptr[0]) : 0;
    f.order = h.flow_order[flow_dir].as<int32_t>();
    f.dep_ptr = h.flow_dep_ptr[flow_dir].as<int32_t>();
    f.dep_idx = h.flow_dep_idx[flow_dir].as<int32_t>();
    f.done = h.flow_done.as<int32_t>();
    f.counter = h.flow_counter.as<unsigned long long>();
    f.base = h.flow_base;
    f.target = f.roles * (h.flow_seq + 1);
    // one workgroup per task; each takes one counter value
    if (h.kev0)
      hipExtLaunchKernelGGL(fk, dim3((unsigned)f.ntasks), dim3(NW * 64), (uint32_t)lds, s, h.kev0, h.kev1, 0u, a, f);
    else
      hipLaunchKernelGGL(fk, dim3((unsigned)f.ntasks), dim3(NW * 64), lds, s, a, f);
    DDG_HIP(hipGetLastError());
    h.flow_base += f.ntasks;
    h.flow_seq += 1;
    return;
  }
  auto kern = k_sweep<FT, AT, T, NW, TPW, SL>;
  if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (residual) {
    with_lanes(h.lpr, [&](auto Lc) {
      constexpr int L = decltype(Lc)::value;
      hipLaunchKernelGGL(k_local_residual<L>, dim3((unsigned)(((int64_t)S.max_set * L + 255) / 256), (unsigned)nsub),
                         dim3(256), 0, s, st, a.sub_inst, a.subs, a.set_ptr, a.set_idx, a.rp, a.ci, a.val,
                         dia_view(h), r, e, a.e_zero, h.ws.bres);
    });
    DDG_HIP(hipGetLastError());
    return;
  }
  const unsigned grid = a.twisted ? (unsigned)(16 * ((nsub + 7) / 8)) : (unsigned)nsub;
  if constexpr (SL) {
    // grouped launch: when the colour leaves CUs idle and the local problems have
    // levels of at least grp_split rounds, G workgroups per chain (every workgroup
    // of the launch resident at once, one per CU)
    const int max_rounds = (tiles_for(S.max_blk, T) + NW * TPW - 1) / (NW * TPW);
    int G = 1;
    if (h.grp_max > 1 && nsub <= h.grp_slots && max_rounds >= h.grp_split)
      G = std::min(h.grp_max, h.n_cu / (int)grid);
    if (G > 1) {
      h.grp_used = std::max(h.grp_used, G);
      a.groups = G;
      a.split_rounds = h.grp_split;
      auto gk = k_sweep<FT, AT, T, NW, TPW, SL, true>;
      if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)gk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      if (h.kev0)
        hipExtLaunchKernelGGL(gk, dim3(grid * G), dim3(NW * 64), (uint32_t)lds, s, h.kev0, h.kev1, 0u, a);
      else
        hipLaunchKernelGGL(gk, dim3(grid * G), dim3(NW * 64), lds, s, a);
      DDG_HIP(hipGetLastError());
      return;
    }
  }
  if (h.kev0)
    hipExtLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), (uint32_t)lds, s, h.kev0, h.kev1, 0u, a);
  else
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NW * 64), lds, s, a);
  DDG_HIP(hipGetLastError());
}

// The local-solve launch shapes: (waves, tiles per wave per round) keep the register
// ring within 128 VGPRs at 16 waves or 256 at 8 waves, without spills (the sliced
// path's prefetched couplings take a few registers of their own).  fn is called with
// a SweepCfg of the handle's factor precision, coupling layout and tile edge.
template <class FT_, class AT_, int T_, int NW_, int TPW_, bool SL_>
struct SweepCfg {
  using FT = FT_;
  using AT = AT_;
  static constexpr int T = T_, NW = NW_, TPW = TPW_;
  static constexpr bool SL = SL_;
};

template <class FT, class AT, bool SL, class Fn>
void with_cfg_tile(int tile, Fn&& fn) {
  switch (tile) {
    case 16: fn(SweepCfg<FT, AT, 16, 4, 4, SL>{}); break;
    case 32:
      if constexpr (sizeof(FT) == 8) fn(SweepCfg<FT, AT, 32, 8, 4, SL>{});
      else if constexpr (SL) fn(SweepCfg<FT, AT, 32, 8, 7, SL>{});
      else fn(SweepCfg<FT, AT, 32, 8, 8, SL>{});
      break;
    default:
      if constexpr (sizeof(FT) == 8) fn(SweepCfg<FT, AT, 64, 8, 1, SL>{});
      else fn(SweepCfg<FT, AT, 64, 8, 2, SL>{});
      break;
  }
}

template <class FT, class AT, class Fn>
void with_cfg_layout(const Handle& h, Fn&& fn) {
  if (h.S.sliced) with_cfg_tile<FT, AT, true>(h.S.tile, fn);
  else with_cfg_tile<FT, AT, false>(h.S.tile, fn);
}

template <class Fn>
void with_sweep_cfg(const Handle& h, Fn&& fn) {
  switch (h.opt.precision) {
    case DDG_MIXED_FP32: with_cfg_layout<float, float>(h, fn); break;
    case DDG_MIXED_BF16: with_cfg_layout<__hip_bfloat16, float>(h, fn); break;
    default: with_cfg_layout<double, double>(h, fn); break;
  }
}

}  // namespace

namespace {

// SSOR smoothing of the subdomains of one colour (DDG_LOCAL_SSOR, Section 7's
// inexact variant): one workgroup per subdomain, the local right-hand side
// b = (r - A e)[set] (the local-residual kernel's output) and the iterate x kept
// on chip.  Each relaxation x_r += omega (b_r - (A_i x)_r) / a_rr covers the rows
// of one local colour at once (they are not coupled), colours ascending then
// descending, `sweeps` times from x = 0; then e[set] += x.
constexpr int kSsorThreads = 512;

__global__ void __launch_bounds__(kSsorThreads) k_ssor(
    const int32_t* __restrict__ subs, const int64_t* __restrict__ set_ptr, const int32_t* __restrict__ set_idx,
    const int64_t* __restrict__ ss_ptr, const int32_t* __restrict__ ss_col, const double* __restrict__ ss_val,
    const double* __restrict__ ss_diag, const int32_t* __restrict__ ss_perm, const int32_t* __restrict__ ss_cptr,
    const int32_t* __restrict__ ss_coff, const double* __restrict__ bres, double* __restrict__ e,
    const CgState* st, const int32_t* __restrict__ sub_inst, double omega, int sweeps, int ld) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* x = reinterpret_cast<double*>(smem_raw);
  double* b = x + ld;
  const int sub = subs[blockIdx.x];
  if (st && st[sub_inst[sub]].done) return;
  const int64_t s0 = set_ptr[sub];
  const int ni = (int)(set_ptr[sub + 1] - s0);
  for (int j = threadIdx.x; j < ni; j += kSsorThreads) {
    x[j] = 0.0;
    b[j] = bres[s0 + j];
  }
  __syncthreads();
  const int c0 = ss_cptr[sub];
  const int nc = ss_cptr[sub + 1] - c0 - 1;
  for (int sw = 0; sw < sweeps; ++sw) {
    for (int q = 0; q < 2 * nc; ++q) {
      const int c = q < nc ? q : 2 * nc - 1 - q;
      const int t1 = ss_coff[c0 + c + 1];
      for (int t = ss_coff[c0 + c] + threadIdx.x; t < t1; t += kSsorThreads) {
        const int rl = ss_perm[s0 + t];
        const int64_t g = s0 + rl;
        double acc = b[rl];
        for (int64_t k = ss_ptr[g]; k < ss_ptr[g + 1]; ++k) acc -= ss_val[k] * x[ss_col[k]];
        x[rl] += omega * acc / ss_diag[g];
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < ni; j += kSsorThreads) e[set_idx[s0 + j]] += x[j];
}

// One colour phase with SSOR smoothing: its local-residual kernel, or its smoothing.
void launch_ssor_phase(const Handle& h, int colour, const double* r, double* e, bool e_zero, const CgState* st,
                       hipStream_t s, bool residual) {
  const Symbolic& S = h.S;
  const int nsub = S.colour_ptr[colour + 1] - S.colour_ptr[colour];
  if (nsub == 0) return;
  const int32_t* subs = h.colour_subs.as<int32_t>() + S.colour_ptr[colour];
  if (residual) {
    with_lanes(h.lpr, [&](auto Lc) {
      constexpr int L = decltype(Lc)::value;
      hipLaunchKernelGGL(k_local_residual<L>, dim3((unsigned)(((int64_t)S.max_set * L + 255) / 256), (unsigned)nsub),
                         dim3(256), 0, s, st, h.sub_inst.as<int32_t>(), subs, h.set_ptr.as<int64_t>(),
                         h.set_idx.as<int32_t>(), h.rowptr.as<int64_t>(), h.col.as<int32_t>(), h.val.as<double>(),
                         dia_view(h), r, e, e_zero ? 1 : 0, h.ws.bres);
    });
    DDG_HIP(hipGetLastError());
    return;
  }
  const int ld = (S.max_set + 1) & ~1;
  const size_t lds = (size_t)2 * ld * sizeof(double);
  DDG_REQUIRE(lds + 1024 <= (size_t)h.dev_lds_limit, DDG_ERR_UNSUPPORTED,
              "expanded set too large for on-chip SSOR smoothing (" + std::to_string(S.max_set) + " rows)");
  if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)k_ssor, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  if (h.kev0)
    hipExtLaunchKernelGGL(k_ssor, dim3((unsigned)nsub), dim3(kSsorThreads), (uint32_t)lds, s, h.kev0, h.kev1, 0u,
                          subs, h.set_ptr.as<int64_t>(), h.set_idx.as<int32_t>(), h.ss_ptr.as<int64_t>(),
                          h.ss_col.as<int32_t>(), h.ss_val.as<double>(), h.ss_diag.as<double>(),
                          h.ss_perm.as<int32_t>(), h.ss_cptr.as<int32_t>(), h.ss_coff.as<int32_t>(), h.ws.bres, e, st,
                          h.sub_inst.as<int32_t>(), h.opt.ssor_omega, h.opt.ssor_sweeps, ld);
  else
    hipLaunchKernelGGL(k_ssor, dim3((unsigned)nsub), dim3(kSsorThreads), lds, s, subs, h.set_ptr.as<int64_t>(),
                       h.set_idx.as<int32_t>(), h.ss_ptr.as<int64_t>(), h.ss_col.as<int32_t>(),
                       h.ss_val.as<double>(), h.ss_diag.as<double>(), h.ss_perm.as<int32_t>(),
                       h.ss_cptr.as<int32_t>(), h.ss_coff.as<int32_t>(), h.ws.bres, e, st, h.sub_inst.as<int32_t>(),
                       h.opt.ssor_omega, h.opt.ssor_sweeps, ld);
  DDG_HIP(hipGetLastError());
}

}  // namespace

// residual = true: launch only the local-residual kernel of the colour; false: the local solves.
void launch_sweep(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                  const CgState* st, hipStream_t s, bool res) {
  if (h.ssor) {
    launch_ssor_phase(h, colour, r, e, e_zero, st, s, res);
    return;
  }
  with_sweep_cfg(h, [&](auto c) {
    using C = decltype(c);
    launch_sweep_cfg<typename C::FT, typename C::AT, C::T, C::NW, C::TPW, C::SL>(h, colour, r, e, e_zero, st, s,
                                                                                 res, -1);
  });
}

// dir 0: the ascending sweep (e is zero on entry); 1: the descending sweep.
void launch_sweep_flow(Handle& h, int dir, const double* r, double* e, const CgState* st, hipStream_t s) {
  DDG_REQUIRE(h.flow_ok, DDG_ERR_HIP, "internal: persistent sweep not prepared");
  with_sweep_cfg(h, [&](auto c) {
    using C = decltype(c);
    launch_sweep_cfg<typename C::FT, typename C::AT, C::T, C::NW, C::TPW, C::SL>(h, 0, r, e, dir == 0, st, s, false,
                                                                                 dir);
  });
}


// ---------------------------------------------------------------------------
// Persistent batched solve (DDG_SCHEDULE_PERSISTENT): the whole PCG of every
// system of the handle in one launch.  Workgroups take tasks from a device ring
// in order.  A task is one chunk of rows, one subdomain's local solve, one
// restriction chunk, a group of coarse tiles or one system's scalar step.  Each
// system walks its own sequence of phases, the steps of the one-launch-per-step
// driver in the same order: e = 0, the colours of the pre-sweep, restriction,
// coarse solve, prolongation, the colours of the post-sweep, r.z, rho and beta,
// the direction update, q = A p with p.q, alpha, the x and r update with r.r,
// the convergence test.  The workgroup that finishes the last task of a phase
// enqueues the next phase of that system, so systems advance and stop
// independently.  Every task runs the device body of the per-step kernels on
// the same data and rows, so every value is the same bit for bit.  No task
// waits for another task: a workgroup only waits for the ring slot it claimed to
// be published (bounded by a wall-clock limit), and it leaves once every system
// has stopped.
namespace {

enum PTask : int32_t {
  PT_EXIT = 0, PT_INIT, PT_INIT_S, PT_ZERO, PT_SWEEP_F, PT_RESTRICT, PT_RSUM, PT_SYMV, PT_CSUM, PT_PROLONG,
  PT_SWEEP_B, PT_DOT, PT_RHO, PT_XPBY, PT_SPMV, PT_ALPHA, PT_AXPY, PT_CONV
};

// A ring slot is one 64-bit word, written and read whole: kind (5 bits), aux (7: the
// colour of a sweep task, the first-iteration flag of r.z and rho), system (16),
// task index within the phase (21), and the lap of the ring position (15), which
// tells a published slot from the one of the previous lap.  Empty slots hold ~0.
constexpr int kPsTagShift = 49;
constexpr uint64_t kPsTagMask = 0x7FFF;
constexpr int kPsRowsPerTask = 256;   // coarse entries or rows per summation task

__host__ __device__ inline uint64_t ps_word(int kind, int aux, int sys, int idx, uint64_t lap) {
  return (uint64_t)kind | ((uint64_t)aux << 5) | ((uint64_t)sys << 12) | ((uint64_t)idx << 28) |
         ((lap & kPsTagMask) << kPsTagShift);
}

struct PSys {
  int32_t phase;    // PTask of the running phase
  int32_t colour;   // colour of a sweep phase
  int32_t count;    // tasks of the running phase
  int32_t first;    // 1 until the first r.z and rho have run
};

struct PsCtl {
  unsigned long long head;   // next ring position to claim
  unsigned long long tail;   // next ring position to allocate
  int32_t all_done;          // every system has stopped (or the launch gave up)
  int32_t remaining;         // systems not yet stopped
  int32_t next_sys;          // position in the admission order of the next system to start
};

struct PersistArgs {
  uint64_t* ring;
  uint64_t mask;
  int32_t log2size;
  PsCtl* ctl;
  const int32_t* order;      // admission order of the systems (smallest first)
  int32_t nb;
  PSys* sys;
  int32_t* cnt;              // per system: finished tasks of the running phase
  int32_t* err;
  uint64_t wait_ticks;       // wall-clock limit of one wait for a slot
  // CG
  CgState* st;
  SegMap m;
  Hist hist;
  double rtol;
  int32_t max_iter;
  int32_t pr;                // Polak-Ribiere direction update
  const double* f;
  double *x, *r, *p, *q, *z;
  double *part, *part2;
  const int64_t* rp;
  const int32_t* ci;
  const double* val;
  DiaView D;
  int32_t lpr;
  // sweeps: per (system, colour) subdomain lists
  const int32_t* ps_ptr;     // nb * C + 1
  const int32_t* ps_sub;
  int32_t C;
  // coarse correction
  int32_t has_coarse;
  const int32_t* sub_off;    // nb + 1
  const int32_t* sub_inst;
  const int64_t* own_ptr;
  const int32_t* own_idx;
  const int32_t* kcnt;
  const int64_t* koff;
  const int32_t* part_id;    // subdomain of every row
  const int32_t* qpos;       // position of every row in the own-row order
  const double* Qo;          // the basis in the own-row layout (q_own_at)
  int32_t kq;
  int32_t nch, rch;
  double* rpart;
  double* b0;
  double* y;
  const int64_t* tile_base;
  const int64_t* cblk_off;
  const int32_t* cblk_n;
  const double* tiles;
  double *rowpart, *colpart;
};

template <class Fn>
__device__ inline void with_lanes_dev(int L, Fn&& f) {
  switch (L) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

// tasks of phase ph (colour c) of system b; NW tiles per coarse-GEMV task
__host__ __device__ inline int32_t ps_count(int ph, int c, int chunks, const int32_t* ps_ptr, int b, int C,
                                            int nsub, int nch, int64_t ntiles, int64_t crows, int NW) {
  switch (ph) {
    case PT_INIT: case PT_ZERO: case PT_PROLONG: case PT_DOT: case PT_XPBY: case PT_SPMV: case PT_AXPY:
      return chunks;
    case PT_SWEEP_F: case PT_SWEEP_B: return ps_ptr[b * C + c + 1] - ps_ptr[b * C + c];
    case PT_RESTRICT: return nsub * nch;
    case PT_RSUM: return (nsub * 32 + kPsRowsPerTask - 1) / kPsRowsPerTask;
    case PT_SYMV: return (int32_t)((ntiles + NW - 1) / NW);
    case PT_CSUM: return (int32_t)((crows + kPsRowsPerTask - 1) / kPsRowsPerTask);
    default: return 1;
  }
}

template <int NW>
__device__ inline int32_t p_count(const PersistArgs& P, int b, int ph, int c) {
  return ps_count(ph, c, P.m.ptr[b + 1] - P.m.ptr[b], P.ps_ptr, b, P.C, P.sub_off[b + 1] - P.sub_off[b], P.nch,
                  P.has_coarse ? P.tile_base[b + 1] - P.tile_base[b] : 0,
                  P.has_coarse ? P.cblk_off[b + 1] - P.cblk_off[b] : 0, NW);
}

// The phase after (ph, c) of system b, skipping phases without tasks; PT_EXIT once
// the system has stopped.  first: the first r.z (after the first preconditioner).
template <int NW>
__device__ inline void p_next(const PersistArgs& P, int b, int& ph, int& c, int first) {
  const bool coarse = P.has_coarse && P.cblk_n[b] > 0;
  const bool done = P.st[b].done != 0;
  for (;;) {
    switch (ph) {
      case PT_INIT: ph = PT_INIT_S; break;
      case PT_INIT_S: ph = done ? PT_EXIT : PT_ZERO; break;
      case PT_ZERO: ph = PT_SWEEP_F; c = 0; break;
      case PT_SWEEP_F:
        if (c + 1 < P.C) ++c;
        else if (coarse) ph = PT_RESTRICT;
        else { ph = PT_SWEEP_B; c = P.C - 1; }
        break;
      case PT_RESTRICT: ph = PT_RSUM; break;
      case PT_RSUM: ph = PT_SYMV; break;
      case PT_SYMV: ph = PT_CSUM; break;
      case PT_CSUM: ph = PT_PROLONG; break;
      case PT_PROLONG: ph = PT_SWEEP_B; c = P.C - 1; break;
      case PT_SWEEP_B:
        if (c > 0) --c;
        else ph = PT_DOT;
        break;
      case PT_DOT: ph = PT_RHO; break;
      case PT_RHO: ph = done ? PT_EXIT : (first ? PT_SPMV : PT_XPBY); break;
      case PT_XPBY: ph = PT_SPMV; break;
      case PT_SPMV: ph = PT_ALPHA; break;
      case PT_ALPHA: ph = done ? PT_EXIT : PT_AXPY; break;
      case PT_AXPY: ph = PT_CONV; break;
      case PT_CONV: ph = done ? PT_EXIT : PT_ZERO; break;
      default: ph = PT_EXIT; break;
    }
    if (ph == PT_EXIT || p_count<NW>(P, b, ph, c) > 0) return;
  }
}

// At least two waves per SIMD (three at tile edge 16): the task bodies together would
// otherwise take every register of the SIMD at the 256-thread shape and leave one
// workgroup per CU (no reference to the by-value arguments may reach a body that is
// not inlined, or they are copied to private memory).  At edge 16 the third wave is
// worth its spills (batch of 256: 206 -> 201 ms per solve); the wider tiles' sweep
// bodies alone need more than a third of the register file.
template <class FT, class AT, int T, int NW, int TPW, bool SL>
__global__ void __launch_bounds__(NW * 64, T == 16 ? 3 : 2) k_persist(SweepArgs a, PersistArgs P) {
  constexpr int NT = NW * 64;
  __shared__ int32_t s_task[5];
  __shared__ int32_t s_next[4];
  __shared__ unsigned long long s_base;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) {
      const unsigned long long pos = atomicAdd(&P.ctl->head, 1ull);
      const uint64_t want = (pos >> P.log2size) & kPsTagMask;
      const uint64_t* sl = P.ring + (pos & P.mask);
      int kind = PT_EXIT;
      const uint64_t t0 = (uint64_t)wall_clock64();
      for (int spin = 1;; ++spin) {
        const uint64_t v = __hip_atomic_load(sl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((v >> kPsTagShift) == want) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          wait_vm();
          kind = (int)(v & 31);
          const int b = (int)((v >> 12) & 0xFFFF);
          s_task[1] = b;
          s_task[2] = (int)((v >> 28) & 0x1FFFFF);
          s_task[3] = (int)((v >> 5) & 127);
          // the phase's task count, read while this task is unfinished: the last
          // finisher replaces it only after every task of the phase has counted itself
          s_task[4] = __hip_atomic_load(&P.sys[b].count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        if (__hip_atomic_load(&P.ctl->all_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        __builtin_amdgcn_s_sleep(2);
        if ((spin & 255) == 0 && (uint64_t)wall_clock64() - t0 > P.wait_ticks) {
          if (atomicCAS(P.err, 0, DDG_ERR_HIP) == 0) {
            P.err[1] = -1;
            P.err[2] = -10;
          }
          __hip_atomic_store(&P.ctl->all_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      s_task[0] = kind;
    }
    __syncthreads();
    const int kind = s_task[0], b = s_task[1], idx = s_task[2], aux = s_task[3], need = s_task[4];
    __syncthreads();
    if (kind == PT_EXIT) return;
    const int g = P.m.ptr[b] + idx;   // chunk of rows (chunk tasks)
    switch (kind) {
      case PT_INIT: d_cg_init(P.m, g, P.f, P.x, P.r, P.part); break;
      case PT_INIT_S: d_cg_init_scalar(P.st, P.m, b, P.part, P.rtol, P.max_iter, P.hist); break;
      case PT_ZERO: d_zero(P.m, g, P.z); break;
      case PT_SWEEP_F:
      case PT_SWEEP_B: {
        const int sub = P.ps_sub[P.ps_ptr[b * P.C + aux] + idx];
        sweep_task<FT, AT, T, NW, TPW, SL, true>(a, sub, 0, sub, kind == PT_SWEEP_F && aux == 0);
        break;
      }
      case PT_RESTRICT: {
        const int i = P.sub_off[b] + idx / P.nch, c = idx % P.nch;
        with_lanes_dev(P.lpr, [&](auto Lc) {
          constexpr int L = decltype(Lc)::value;
          d_coarse_restrict<L, 32>(i, c, P.nch, P.sub_inst, P.own_ptr, P.own_idx, P.kcnt, P.Qo, P.kq, P.rp, P.ci,
                                   P.val, P.D, P.r, P.z, P.rch, P.rpart);
        });
        break;
      }
      case PT_RSUM: {
        const int i0 = P.sub_off[b], ne = (P.sub_off[b + 1] - i0) * 32;
        const int e = idx * kPsRowsPerTask + tid;
        if (tid < kPsRowsPerTask && e < ne) d_coarse_restrict_sum_entry(i0 + e / 32, e % 32, P.kcnt, P.koff, P.rpart, P.nch, 32, P.b0);
        break;
      }
      case PT_SYMV: {
        const int64_t t = P.tile_base[b] + (int64_t)idx * NW + (tid >> 6);
        if (t < P.tile_base[b + 1]) d_coarse_symv_tile(t, b, P.tile_base, P.cblk_off, P.tiles, P.b0, P.rowpart, P.colpart);
        break;
      }
      case PT_CSUM: {
        const int64_t row = P.cblk_off[b] + (int64_t)idx * kPsRowsPerTask + tid;
        if (tid < kPsRowsPerTask && row < P.cblk_off[b + 1])
          d_coarse_sum_row(row, b, P.tile_base, P.cblk_off, P.rowpart, P.colpart, P.y);
        break;
      }
      case PT_PROLONG:
        for (int64_t row = P.m.lo[g] + tid; row < P.m.hi[g]; row += NT)
          d_coarse_prolong_row<32>(row, P.qpos[row], nullptr, P.sub_inst, P.part_id, P.kcnt, P.koff, P.Qo, P.kq,
                                   P.y, P.z);
        break;
      case PT_DOT:
        if (aux) d_copy_dot(P.m, g, P.r, P.z, P.p, P.part);
        else if (P.pr) d_dot2(P.m, g, P.r, P.z, P.q, P.part, P.part2);
        else d_dot(P.m, g, P.r, P.z, P.part);
        break;
      case PT_RHO: d_rho_scalar(P.st, P.m, b, P.part, P.pr && !aux ? P.part2 : nullptr, aux, P.hist); break;
      case PT_XPBY: d_xpby(P.st + b, P.m, g, P.z, P.p); break;
      case PT_SPMV:
        with_lanes_dev(P.lpr, [&](auto Lc) {
          constexpr int L = decltype(Lc)::value;
          d_spmv_dot<L>(P.m, g, P.rp, P.ci, P.val, P.D, P.p, P.q, P.part);
        });
        break;
      case PT_ALPHA: d_alpha_scalar(P.st, P.m, b, P.part, P.hist); break;
      case PT_AXPY: d_axpy2_dot(P.st + b, P.m, g, P.x, P.r, P.p, P.q, P.part); break;
      case PT_CONV: d_conv_scalar(P.st, P.m, b, P.part, P.hist); break;
      default: break;
    }
    // completion: publish this task's stores and count it; the last task of the
    // phase moves its system on
    wait_vm();
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      wait_vm();
      const int32_t finished = __hip_atomic_fetch_add(P.cnt + b, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
      int n_next = 0;
      if (finished == need) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        wait_vm();
        PSys s = P.sys[b];
        int ph = s.phase, c = s.colour;
        const int first = s.first;
        p_next<NW>(P, b, ph, c, first);
        if (s.phase == PT_RHO) s.first = 0;
        if (ph == PT_EXIT) {
          if (__hip_atomic_fetch_add(&P.ctl->remaining, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1)
            __hip_atomic_store(&P.ctl->all_done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // the stopped system's place goes to the next system in the admission order
          const int q = __hip_atomic_fetch_add(&P.ctl->next_sys, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (q < P.nb) {
            const int b2 = P.order[q];
            n_next = P.m.ptr[b2 + 1] - P.m.ptr[b2];   // its first phase (PT_INIT, state from the reset)
            s_base = atomicAdd(&P.ctl->tail, (unsigned long long)n_next);
            s_next[1] = PT_INIT;
            s_next[2] = 0;
            s_next[3] = b2;
          }
        } else {
          n_next = p_count<NW>(P, b, ph, c);
          s.phase = ph;
          s.colour = c;
          s.count = n_next;
          P.sys[b] = s;
          __hip_atomic_store(P.cnt + b, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          // the state is in memory before any task of the next phase can be claimed
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
          wait_vm();
          s_base = atomicAdd(&P.ctl->tail, (unsigned long long)n_next);
          s_next[1] = ph;
          s_next[2] = (ph == PT_SWEEP_F || ph == PT_SWEEP_B) ? c : ((ph == PT_DOT || ph == PT_RHO) ? first : 0);
          s_next[3] = b;
        }
      }
      s_next[0] = n_next;
    }
    __syncthreads();
    const int n_next = s_next[0];
    if (n_next > 0) {
      const int ph = s_next[1], aux2 = s_next[2], tb = s_next[3];
      const unsigned long long base = s_base;
      for (int t = tid; t < n_next; t += NT) {
        const unsigned long long pos = base + (unsigned long long)t;
        __hip_atomic_store(P.ring + (pos & P.mask), ps_word(ph, aux2, tb, t, pos >> P.log2size), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

// ring reset: the initial tasks (PT_INIT of every system) at the first positions,
// every other slot empty; the per-system states and counts from their initial values
__global__ void k_persist_reset(uint64_t* __restrict__ ring, int64_t size, const uint64_t* __restrict__ init,
                                int32_t n_init, PSys* __restrict__ sys, const PSys* __restrict__ sys0,
                                int32_t* __restrict__ cnt, int32_t nb, int32_t n_admit, PsCtl* __restrict__ ctl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < size) ring[i] = i < n_init ? init[i] : ~0ull;
  if (i < nb) {
    sys[i] = sys0[i];
    cnt[i] = 0;
  }
  if (i == 0) {
    ctl->head = 0;
    ctl->tail = (unsigned long long)n_init;
    ctl->all_done = 0;
    ctl->remaining = nb;
    ctl->next_sys = n_admit;
  }
}

template <class FT, class AT, int T, int NW, int TPW, bool SL>
void launch_persist_cfg(Handle& h, const double* f, double* x, hipStream_t s) {
  const Symbolic& S = h.S;
  SweepArgs a;
  const size_t lds = build_sweep_args<FT, AT, T, NW, TPW, SL>(h, h.colour_subs.as<int32_t>(), S.n_parts,
                                                              h.r.as<double>(), h.z.as<double>(), false, nullptr, a);
  auto kern = k_persist<FT, AT, T, NW, TPW, SL>;
  if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int occ = 0;
  DDG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, NW * 64, lds));
  const int64_t grid = (int64_t)h.n_cu * std::max(1, occ);
  // ring: at least twice the most tasks that can be outstanding at once plus the grid
  // (a slot is reused only after the whole ring has been claimed since), a power of two
  int32_t lg = 10;
  while (((int64_t)1 << lg) < 2 * (h.ps_omax + grid)) ++lg;
  DDG_REQUIRE(lg <= 30, DDG_ERR_UNSUPPORTED, "persistent schedule: too many tasks");
  const int64_t size = (int64_t)1 << lg;
  if (h.ps_ring.bytes < (size_t)size * sizeof(uint64_t)) h.ps_ring.alloc((size_t)size * sizeof(uint64_t));
  hipLaunchKernelGGL(k_persist_reset, dim3((unsigned)((std::max<int64_t>(size, h.nb) + 255) / 256)), dim3(256), 0, s,
                     h.ps_ring.as<uint64_t>(), size, h.ps_init.as<uint64_t>(), h.ps_ninit, h.ps_sys.as<PSys>(),
                     h.ps_sys0.as<PSys>(), h.ps_cnt.as<int32_t>(), h.nb, h.ps_admit, h.ps_ctl.as<PsCtl>());
  PersistArgs P{};
  P.ring = h.ps_ring.as<uint64_t>();
  P.mask = (uint64_t)size - 1;
  P.log2size = lg;
  P.ctl = h.ps_ctl.as<PsCtl>();
  P.order = h.ps_order.as<int32_t>();
  P.nb = h.nb;
  P.sys = h.ps_sys.as<PSys>();
  P.cnt = h.ps_cnt.as<int32_t>();
  P.err = h.err_flag.as<int32_t>();
  P.wait_ticks = (uint64_t)h.clock_khz * 30000ull;   // 30 s
  P.st = h.cstate.as<CgState>();
  P.m = SegMap{h.wg_seg.as<int32_t>(), h.wg_lo.as<int64_t>(), h.wg_hi.as<int64_t>(), h.seg_wg_ptr_d.as<int32_t>()};
  P.hist = Hist{h.hist.as<double>(), (int64_t)h.opt.max_iter + 1};
  P.rtol = h.opt.rtol;
  P.max_iter = h.opt.max_iter;
  P.pr = h.opt.cg_variant == DDG_CG_POLAK_RIBIERE ? 1 : 0;
  P.f = f;
  P.x = x;
  P.r = h.r.as<double>();
  P.p = h.p.as<double>();
  P.q = h.q.as<double>();
  P.z = h.z.as<double>();
  P.part = h.part_sums.as<double>();
  P.part2 = P.part + h.n_partials;
  P.rp = h.rowptr.as<int64_t>();
  P.ci = h.col.as<int32_t>();
  P.val = h.val.as<double>();
  P.D = dia_view(h);
  P.lpr = h.lpr;
  P.ps_ptr = h.ps_ptr.as<int32_t>();
  P.ps_sub = h.ps_sub.as<int32_t>();
  P.C = S.n_colours;
  P.has_coarse = h.nc > 0 ? 1 : 0;
  P.sub_off = h.ps_suboff.as<int32_t>();
  P.sub_inst = h.sub_inst.as<int32_t>();
  if (h.nc > 0) {
    P.own_ptr = h.own_ptr.as<int64_t>();
    P.own_idx = h.own_idx.as<int32_t>();
    P.kcnt = h.kcnt_d.as<int32_t>();
    P.koff = h.koff_d.as<int64_t>();
    P.part_id = h.part.as<int32_t>();
    P.qpos = h.qpos.as<int32_t>();
    P.Qo = h.Qo.as<double>();
    P.kq = h.k;
    P.nch = h.nch;
    P.rch = h.rch;
    P.rpart = h.ws.rpart;
    P.b0 = h.ws.cy;
    P.y = h.ws.cy + h.nc_pad;
    P.tile_base = h.tile_base_d.as<int64_t>();
    P.cblk_off = h.cblk_off_d.as<int64_t>();
    P.cblk_n = h.cblk_n_d.as<int32_t>();
    P.tiles = h.A0inv_t.as<double>();
    P.rowpart = h.ws.cpart;
    P.colpart = h.ws.cpart + h.ntiles * 64;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(NW * 64), lds, s, a, P);
  DDG_HIP(hipGetLastError());
}

}  // namespace

// Host tables of the persistent schedule (per system and colour, its subdomains in
// the colour lists' order; the initial ring words and states; the most tasks that
// can be outstanding at once).
void prepare_persist(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  const int32_t nb = h.nb, C = S.n_colours;
  DDG_REQUIRE(!h.three_level && !h.ssor && !h.ic && h.k <= 32, DDG_ERR_UNSUPPORTED,
              "persistent schedule: needs exact local solves, the explicit coarse inverse, two levels and at "
              "most 32 generating vectors");
  DDG_REQUIRE(C < 128 && nb < 65536, DDG_ERR_UNSUPPORTED, "persistent schedule: at most 127 colours and 65535 systems");
  std::vector<int32_t> sub_sys(S.n_parts);
  for (int32_t b = 0; b < nb; ++b)
    for (int32_t i = h.sub_off[b]; i < h.sub_off[b + 1]; ++i) sub_sys[i] = b;
  std::vector<std::vector<int32_t>> lists((size_t)nb * C);
  for (int32_t c = 0; c < C; ++c)
    for (int32_t t = S.colour_ptr[c]; t < S.colour_ptr[c + 1]; ++t) {
      const int32_t sub = S.colour_subs[t];
      lists[(size_t)sub_sys[sub] * C + c].push_back(sub);
    }
  std::vector<int32_t> ptr((size_t)nb * C + 1, 0), subs;
  subs.reserve(S.n_parts);
  for (size_t q = 0; q < lists.size(); ++q) {
    subs.insert(subs.end(), lists[q].begin(), lists[q].end());
    ptr[q + 1] = (int32_t)subs.size();
  }
  // admission: systems start smallest first; enough of them at once for about sixteen
  // subdomains per CU (a system offers only its current colour's subdomains as sweep
  // tasks, so fewer leave workgroups without work), and each stopped system hands its
  // place to the next one
  std::vector<int32_t> order(nb);
  for (int32_t b = 0; b < nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    return h.seg_off[x + 1] - h.seg_off[x] < h.seg_off[y + 1] - h.seg_off[y];
  });
  int32_t admit = 0;
  for (int64_t subs = 0; admit < nb && subs < 16 * (int64_t)h.n_cu; ++admit)
    subs += h.sub_off[order[admit] + 1] - h.sub_off[order[admit]];
  std::vector<uint64_t> init;
  std::vector<PSys> sys0(nb);
  int64_t omax = 0;
  for (int32_t b = 0; b < nb; ++b) {
    const int32_t chunks = h.seg_wg_ptr[b + 1] - h.seg_wg_ptr[b];
    const int32_t nsub = h.sub_off[b + 1] - h.sub_off[b];
    const int64_t ntiles = h.nc > 0 ? h.tile_base[b + 1] - h.tile_base[b] : 0;
    const int64_t crows = h.nc > 0 ? h.cblk_off[b + 1] - h.cblk_off[b] : 0;
    int32_t most = 0;
    for (int ph = PT_INIT; ph <= PT_CONV; ++ph)
      for (int c = 0; c < ((ph == PT_SWEEP_F || ph == PT_SWEEP_B) ? C : 1); ++c)
        most = std::max(most, ps_count(ph, c, chunks, ptr.data(), b, C, nsub, h.nch, ntiles, crows, 4));
    DDG_REQUIRE(most < (1 << 21), DDG_ERR_UNSUPPORTED, "persistent schedule: more than 2^21 tasks in one phase");
    omax += most;
    sys0[b] = PSys{PT_INIT, 0, chunks, 1};
  }
  for (int32_t q = 0; q < admit; ++q) {
    const int32_t b = order[q];
    for (int32_t t = 0; t < h.seg_wg_ptr[b + 1] - h.seg_wg_ptr[b]; ++t) init.push_back(ps_word(PT_INIT, 0, b, t, 0));
  }
  h.ps_omax = omax;
  h.ps_ninit = (int32_t)init.size();
  h.ps_admit = admit;
  h.ps_order.upload(order, s);
  h.ps_ptr.upload(ptr, s);
  h.ps_sub.upload(subs, s);
  h.ps_suboff.upload(h.sub_off, s);
  h.ps_init.upload(init, s);
  h.ps_sys0.upload(sys0, s);
  h.ps_sys.alloc((size_t)nb * sizeof(PSys));
  h.ps_cnt.alloc((size_t)nb * sizeof(int32_t));
  h.ps_ctl.alloc(sizeof(PsCtl));
}

// The whole solve of every system in one launch (schedule DDG_SCHEDULE_PERSISTENT).
void launch_persist(Handle& h, const double* f, double* x, hipStream_t s) {
  DDG_REQUIRE(h.persist, DDG_ERR_HIP, "internal: persistent schedule not prepared");
  DDG_REQUIRE(h.coarse_refine == 0, DDG_ERR_UNSUPPORTED,
              "persistent schedule: the coarse inverse needs refinement steps (ill-conditioned A0)");
  with_sweep_cfg(h, [&](auto c) {
    using Cf = decltype(c);
    launch_persist_cfg<typename Cf::FT, typename Cf::AT, Cf::T, Cf::NW, Cf::TPW, Cf::SL>(h, f, x, s);
  });
}

}  // namespace ddg
