// Setup numerics, all on the device:
//   * coarse basis (Section 4): per subdomain, an orthonormal basis of
//     span F[Omega_i, :] by column-pivoted modified Gram-Schmidt with one
//     re-orthogonalisation pass; a column is discarded when its pivot norm
//     |R_jj| <= rank_tol |R_11| (the paper requires dropping rank-deficient
//     columns without fixing a test);
//   * Galerkin product A0 = R0 A R0^T (Section 4), block (i, j) =
//     Q_i^T A[Omega_i, Omega_j] Q_j for coupled subdomains;
//   * explicit inverse of A0 by blocked Gauss-Jordan (SPD, no pivoting);
//   * local factors (Section 6 exact local solves): for every subdomain the
//     Schur complements S_k of its block-tridiagonal level structure are
//     formed and inverted in float64, then stored as packed lower tiles in
//     the storage precision.
#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

namespace {


// Error record: [0] = code (0 none), [1] = subdomain, [2] = block, [3] = local row
__device__ inline void record_error(int32_t* err, int code, int sub, int blk, int row) {
  if (atomicCAS(err, 0, code) == 0) {
    err[1] = sub;
    err[2] = blk;
    err[3] = row;
  }
}

// Sum `cnt` per-thread values across a 256-thread workgroup; results in out[0..cnt).
template <int NT, int KM>
__device__ inline void multi_sum(double (&acc)[KM], int cnt, double* red /*[NT/64][KM]*/, double* out) {
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m < cnt) {
      double v = wave_sum(acc[m]);
      if ((threadIdx.x & 63) == 0) red[wv * KM + m] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * KM + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Coarse basis

constexpr int kQrThreads = 256;

// KM: capacity of the per-thread column arrays (32, or 80 for up to 80 generating vectors)
template <int KM>
__global__ void __launch_bounds__(kQrThreads) k_coarse_qr(
    const int64_t* __restrict__ own_ptr, const int32_t* __restrict__ own_idx,
    const double* __restrict__ F, int64_t n, int k, double rank_tol, double* __restrict__ work,
    double* __restrict__ Q, int32_t* __restrict__ kcnt, int32_t* __restrict__ err) {
  __shared__ double red[(kQrThreads / 64) * KM];
  __shared__ double sums[KM];
  __shared__ int used[KM];
  __shared__ int pick;
  __shared__ double pick_norm, r11;
  const int i = blockIdx.x;
  const int64_t base = own_ptr[i];
  const int ni = (int)(own_ptr[i + 1] - base);
  double* V = work + base * k;  // column j at V + j*ni
  const int tid = threadIdx.x;
  for (int r = tid; r < ni; r += kQrThreads) {
    const int g = own_idx[base + r];
    for (int j = 0; j < k; ++j) V[(int64_t)j * ni + r] = F[(int64_t)j * n + g];
    for (int j = 0; j < k; ++j) Q[(int64_t)g * k + j] = 0.0;
  }
  if (tid < KM) used[tid] = 0;
  __syncthreads();
  int kept = 0;
  double acc[KM];
  for (int s = 0; s < k; ++s) {
    // residual norms of the unused columns
#pragma unroll
    for (int m = 0; m < KM; ++m) acc[m] = 0.0;
    for (int r = tid; r < ni; r += kQrThreads) {
#pragma unroll
      for (int m = 0; m < KM; ++m)
        if (m < k) {
          double v = V[(int64_t)m * ni + r];
          acc[m] += v * v;
        }
    }
    multi_sum<kQrThreads, KM>(acc, k, red, sums);
    if (tid == 0) {
      int best = -1;
      double bn = -1.0;
      for (int j = 0; j < k; ++j)
        if (!used[j] && sums[j] > bn) {
          bn = sums[j];
          best = j;
        }
      pick = best;
      pick_norm = sqrt(bn);
      if (s == 0) r11 = pick_norm;
    }
    __syncthreads();
    const int jp = pick;
    const double nrm = pick_norm;
    if (s == 0 && !(r11 > 0.0 && isfinite(r11))) {
      if (tid == 0) record_error(err, DDG_ERR_RANK, i, -1, -1);
      break;
    }
    if (!(nrm > rank_tol * r11)) break;
    double* vp = V + (int64_t)jp * ni;
    // re-orthogonalise against the kept basis vectors
    if (kept > 0) {
#pragma unroll
      for (int m = 0; m < KM; ++m) acc[m] = 0.0;
      for (int r = tid; r < ni; r += kQrThreads) {
        const int g = own_idx[base + r];
        const double v = vp[r];
#pragma unroll
        for (int m = 0; m < KM; ++m)
          if (m < kept) acc[m] += Q[(int64_t)g * k + m] * v;
      }
      multi_sum<kQrThreads, KM>(acc, kept, red, sums);
      for (int r = tid; r < ni; r += kQrThreads) {
        const int g = own_idx[base + r];
        double v = vp[r];
        for (int m = 0; m < kept; ++m) v -= sums[m] * Q[(int64_t)g * k + m];
        vp[r] = v;
      }
      __syncthreads();
    }
    acc[0] = 0.0;
    for (int r = tid; r < ni; r += kQrThreads) acc[0] += vp[r] * vp[r];
    multi_sum<kQrThreads, KM>(acc, 1, red, sums);
    const double inv = 1.0 / sqrt(sums[0]);
    for (int r = tid; r < ni; r += kQrThreads) {
      const int g = own_idx[base + r];
      const double qv = vp[r] * inv;
      vp[r] = qv;
      Q[(int64_t)g * k + kept] = qv;
    }
    __syncthreads();
    // modified Gram-Schmidt: project the new direction out of the unused columns
#pragma unroll
    for (int m = 0; m < KM; ++m) acc[m] = 0.0;
    for (int r = tid; r < ni; r += kQrThreads) {
      const double qv = vp[r];
#pragma unroll
      for (int m = 0; m < KM; ++m)
        if (m < k && m != jp && !used[m]) acc[m] += qv * V[(int64_t)m * ni + r];
    }
    multi_sum<kQrThreads, KM>(acc, k, red, sums);
    for (int r = tid; r < ni; r += kQrThreads) {
      const double qv = vp[r];
      for (int m = 0; m < k; ++m)
        if (m != jp && !used[m]) V[(int64_t)m * ni + r] -= sums[m] * qv;
    }
    if (tid == 0) used[jp] = 1;
    __syncthreads();
    ++kept;
  }
  if (tid == 0) kcnt[i] = kept;
}

// ---------------------------------------------------------------------------
// Galerkin product

constexpr int kGalThreads = 256;
constexpr int kGalLds = 48 * 1024;

typedef double gal_d4 __attribute__((ext_vector_type(4)));

// Block row i of A0 = R0 A R0^T (Section 4): for every coupled subdomain j,
//   A0[koff_i + a, koff_j + b] = sum_{g in Omega_i} Q[g, a] (A Q_j)[g, b].
// The rows of Omega_i are taken in chunks: W[r, (s, b)] = (A Q_j)[g_r, b] for a
// group of neighbours s is formed in LDS from the sparse rows, then the dense
// contraction Q_i^T W runs on the FP64 matrix cores (v_mfma_f64_16x16x4: the
// k <= 80 coarse columns of subdomain i are up to five 16-row tiles, each wave
// owns 16-column slabs of the group's (s, b) columns, the chunk rows are the
// reduction dimension).
// MT row tiles of 16 coarse columns (2 for k <= 32, 5 for k <= 80), SL column slabs per wave.
template <int MT, int SL>
__global__ void __launch_bounds__(kGalThreads) k_galerkin(
    const int64_t* __restrict__ own_ptr, const int32_t* __restrict__ own_idx,
    const int32_t* __restrict__ nbr_ptr, const int32_t* __restrict__ nbr_idx,
    const int32_t* __restrict__ part, const int32_t* __restrict__ kcnt,
    const int64_t* __restrict__ koff, const double* __restrict__ Q, int kq,
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ val,
    const int32_t* __restrict__ sub_inst, const int64_t* __restrict__ cblk_off,
    const int32_t* __restrict__ cblk_n, const int64_t* __restrict__ a0_off, double* __restrict__ A0) {
  __shared__ double lds[kGalLds / 8];
  const int i = blockIdx.x;
  // the block row of subdomain i lies in the dense coarse block of its system
  const int sys = sub_inst[i];
  const int64_t c0 = cblk_off[sys], nc = cblk_n[sys];
  double* A0b = A0 + a0_off[sys];
  const int64_t base = own_ptr[i];
  const int ni = (int)(own_ptr[i + 1] - base);
  const int nb0 = nbr_ptr[i];
  const int nnb = nbr_ptr[i + 1] - nb0;
  const int ki = kcnt[i];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mt_n = (kq + 15) / 16;          // row tiles of the k coarse columns of i (<= MT)
  const int slabs_max = MT == 2 ? 4 * (mt_n == 1 ? SL : SL / 2) : 4 * SL;
  const int gmax = max(1, (slabs_max * 16) / kq);
  for (int g0 = 0; g0 < nnb; g0 += gmax) {
    const int gs = min(gmax, nnb - g0);
    const int ncol = gs * kq;
    int ch = kGalLds / (8 * (ncol + kq));
    ch = min(64, ch) & ~3;
    double* Wc = lds;               // [ch][ncol]
    double* Qc = lds + ch * ncol;   // [ch][kq]
    gal_d4 acc[MT][SL];
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int q = 0; q < SL; ++q) acc[m][q] = gal_d4{0.0, 0.0, 0.0, 0.0};
    for (int r0 = 0; r0 < ni; r0 += ch) {
      const int rows = min(ch, ni - r0);
      const int rows4 = (rows + 3) & ~3;
      for (int idx = tid; idx < rows4 * ncol; idx += kGalThreads) Wc[idx] = 0.0;
      __syncthreads();
      // thread (r, b) adds every stored entry of row r into column b of its neighbour's slot
      // (neighbour ids ascending: binary search within the group)
      const int32_t* grp = nbr_idx + nb0 + g0;
      for (int idx = tid; idx < rows * kq; idx += kGalThreads) {
        const int r = idx / kq, b = idx % kq;
        const int g = own_idx[base + r0 + r];
        for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
          const int c = ci[t];
          const int j = part[c];
          int lo = 0, hi = gs;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (grp[mid] < j) lo = mid + 1;
            else hi = mid;
          }
          if (lo < gs && grp[lo] == j) Wc[r * ncol + lo * kq + b] += val[t] * Q[(int64_t)c * kq + b];
        }
      }
      for (int idx = tid; idx < rows4 * kq; idx += kGalThreads) {
        const int r = idx / kq, a = idx % kq;
        Qc[idx] = r < rows ? Q[(int64_t)own_idx[base + r0 + r] * kq + a] : 0.0;
      }
      __syncthreads();
      for (int k0 = 0; k0 < rows4; k0 += 4) {
        const int r = k0 + lk;
        double af[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) {
          const int a = m * 16 + li;
          af[m] = (m < mt_n && a < kq) ? Qc[r * kq + a] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < SL; ++q) {
          const int col = (q * 4 + wave) * 16 + li;
          const double bf = col < ncol ? Wc[r * ncol + col] : 0.0;
#pragma unroll
          for (int m = 0; m < MT; ++m)
            if (m < mt_n) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[m], bf, acc[m][q], 0, 0, 0);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      if (m >= mt_n) continue;
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        const int col = (q * 4 + wave) * 16 + li;
        if (col >= ncol) continue;
        const int sj = col / kq, b = col % kq;
        const int j = nbr_idx[nb0 + g0 + sj];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int a = m * 16 + 4 * e + lk;
          if (a < ki && b < kcnt[j]) A0b[(koff[i] + a - c0) * nc + koff[j] + b - c0] = acc[m][q][e];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Local factorisation (twisted block LDL^T, see kernels_sweep.hip): for each
// subdomain a top chain (levels 0..m-1, couplings to the level below) and a
// bottom chain (levels K-1..m+1, couplings to the level above), then the
// middle level m with both.  Chain step j of every chain of a group runs in
// the same launches ("items", one per active chain):
//   Tm = X_prev C^T            (k_fac_tm)
//   S  = D_k - C Tm            (k_fac_form; the middle level subtracts both sides)
//   S  <- S^{-1}               (the blocked Gauss-Jordan kernels of the coarse
//                               inverse, over all items at once)
//   tiles of S^{-1} -> factor  (k_fac_pack)
// so each panel update of the inversion is spread over thousands of
// workgroups instead of one workgroup per chain.

struct FacItem {
  int32_t cur;     // global block id of the level being factored
  int32_t prev;    // global block id of the coupled level already inverted (-1: none)
  int32_t sub;     // subdomain
  int32_t use_up;  // 0: couplings to the lower level (lo ELL), 1: to the upper level (up ELL)
  int32_t add_d;   // 1: start from the level's diagonal block D_k
  int32_t pad;
  int64_t s_off;   // element offset of S (n x n, row-major) in the scratch
  int64_t x_off;   // element offset of X_prev (bp x bp)
  int64_t t_off;   // element offset of Tm (bp x n)
};

struct FacArgs {
  const FacItem* items;
  const int64_t* set_ptr;
  const int32_t* sub_blk_ptr;
  const int32_t* blk_start;
  const int32_t* blk_size;
  const int64_t* blk_foff;
  const int32_t* lo_col;
  const double* lo_val;
  int32_t cl;
  const int32_t* up_col;
  const double* up_val;
  int32_t cu;
  const int64_t* in_ptr;
  const int32_t* in_col;
  const int64_t* in_pos;
  const double* val;
  double* scratch;
  double* tm;
  void* fac;
};

constexpr int kFacRows = 8;   // rows of the level per workgroup in the formation kernels

// Tm[pp, r] = sum_q X_prev[pp, col_q - bsp] * c_q over the couplings (col_q, c_q) of row r
__global__ void __launch_bounds__(256) k_fac_tm(FacArgs a) {
  const FacItem it = a.items[blockIdx.x];
  if (it.prev < 0) return;
  const int b = a.blk_size[it.cur];
  const int r0 = blockIdx.y * kFacRows;
  if (r0 >= b) return;
  const int bp = a.blk_size[it.prev], bsp = a.blk_start[it.prev];
  const int64_t row0 = a.set_ptr[it.sub] + a.blk_start[it.cur];
  const int cc = it.use_up ? a.cu : a.cl;
  const int32_t* ccol = it.use_up ? a.up_col : a.lo_col;
  const double* cval = it.use_up ? a.up_val : a.lo_val;
  const double* X = a.scratch + it.x_off;
  double* Tm = a.tm + it.t_off;
  const int rows = min(kFacRows, b - r0);
  for (int idx = threadIdx.x; idx < bp * rows; idx += 256) {
    const int pp = idx / rows, r = r0 + idx % rows;
    const int64_t row = row0 + r;
    double acc = 0.0;
    for (int q = 0; q < cc; ++q) {
      const int col = ccol[row * cc + q];
      if (col >= 0) acc += X[(int64_t)pp * bp + (col - bsp)] * cval[row * cc + q];
    }
    Tm[(int64_t)pp * b + r] = acc;
  }
}

// S[r, :] = (add_d ? D_k[r, :] : S[r, :]) - sum_q c_q Tm[col_q - bsp, :]
// A level that starts from D_k and has a coupled level writes 0 - acc first and then adds
// D_k's few stored entries of each row (distinct columns: the input rows are strictly
// increasing): (0 - acc) + d rounds as d - acc does, and S is written once instead of being
// cleared, filled and read back.
__global__ void __launch_bounds__(256) k_fac_form(FacArgs a) {
  const FacItem it = a.items[blockIdx.x];
  const int b = a.blk_size[it.cur];
  const int r0 = blockIdx.y * kFacRows;
  if (r0 >= b) return;
  const int rows = min(kFacRows, b - r0);
  const int bs = a.blk_start[it.cur];
  const int64_t row0 = a.set_ptr[it.sub] + bs;
  double* S = a.scratch + it.s_off;
  if (it.prev < 0) {
    if (!it.add_d) return;
    for (int idx = threadIdx.x; idx < rows * b; idx += 256) S[(int64_t)(r0 + idx / b) * b + idx % b] = 0.0;
    __syncthreads();
    for (int r = threadIdx.x; r < rows; r += 256) {
      const int64_t row = row0 + r0 + r;
      for (int64_t t = a.in_ptr[row]; t < a.in_ptr[row + 1]; ++t)
        S[(int64_t)(r0 + r) * b + (a.in_col[t] - bs)] = a.val[a.in_pos[t]];
    }
    return;
  }
  const int bsp = a.blk_start[it.prev];
  const int cc = it.use_up ? a.cu : a.cl;
  const int32_t* ccol = it.use_up ? a.up_col : a.lo_col;
  const double* cval = it.use_up ? a.up_val : a.lo_val;
  const double* Tm = a.tm + it.t_off;
  for (int idx = threadIdx.x; idx < rows * b; idx += 256) {
    const int r = r0 + idx / b, c = idx % b;
    const int64_t row = row0 + r;
    double acc = 0.0;
    for (int q = 0; q < cc; ++q) {
      const int col = ccol[row * cc + q];
      if (col >= 0) acc += cval[row * cc + q] * Tm[(int64_t)(col - bsp) * b + c];
    }
    double* sp = S + (int64_t)r * b + c;
    if (it.add_d) *sp = 0.0 - acc;
    else *sp -= acc;
  }
  if (!it.add_d) return;
  __syncthreads();
  for (int r = threadIdx.x; r < rows; r += 256) {
    const int64_t row = row0 + r0 + r;
    for (int64_t t = a.in_ptr[row]; t < a.in_ptr[row + 1]; ++t)
      S[(int64_t)(r0 + r) * b + (a.in_col[t] - bs)] += a.val[a.in_pos[t]];
  }
}

// lower T x T tiles of the symmetric n x n matrix S (layout of symv_tile.hpp, diagonal
// tiles compact for compact_diag(T)), converted to FT
template <class FT, int T>
__global__ void __launch_bounds__(256) k_fac_pack(FacArgs a) {
  using G = TileGeom<FT, T>;
  const FacItem it = a.items[blockIdx.x];
  const int b = a.blk_size[it.cur];
  const int nt = (b + T - 1) / T;
  const int ph = last_row_subtiles(b, T);
  const int64_t total = (int64_t)nt * (nt + 1) / 2 * T * T;  // full-tile index space
  const double* S = a.scratch + it.s_off;
  FT* out = static_cast<FT*>(a.fac) + a.blk_foff[it.cur];
  for (int64_t idx = (int64_t)blockIdx.y * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.y * 256) {
    const int t = (int)(idx / (T * T));
    const int within = (int)(idx % (T * T));
    int I, J;
    tile_ij(t, I, J);
    int64_t dst = tile_off<FT, T>(t, I, J, nt, ph);
    const unsigned long long mask = tile_lanes<T>(I, J, nt, ph);
    if (mask != ~0ull) {
      // a compact diagonal tile or a tile of the short last row: only the kept lanes
      // are stored (the others are transposes of stored sub-tiles, or rows past b)
      const int lane = (within / G::E) % 64;
      if (!((mask >> lane) & 1ull)) continue;
      const int c = __builtin_popcountll(mask & ((1ull << lane) - 1ull));
      dst += ((within / (64 * G::E)) * __builtin_popcountll(mask) + c) * G::E + within % G::E;
    } else {
      dst += within;
    }
    int rr, cc;
    tile_rc<FT, T>(within, rr, cc);
    const int row = I * T + rr, col = J * T + cc;
    double v = 0.0;
    if (row < b && col < b) v = (row >= col) ? S[(int64_t)row * b + col] : S[(int64_t)col * b + row];
    out[dst] = Store<FT>::from(v);
  }
}

__global__ void k_gather_vals(const int64_t* __restrict__ pos, const double* __restrict__ val,
                              double* __restrict__ out, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = pos[i] >= 0 ? val[pos[i]] : 0.0;
}

// Sliced coupling values (one workgroup of 64 lanes per slice): entry q of the row
// at lane l takes the row's q-th ELL value, or 0 where the row has fewer couplings
// or the lane lies past the end of its block.  Converted to the sweep's type.
template <class AT>
__global__ void __launch_bounds__(64) k_gather_sliced(const int64_t* __restrict__ sl_row,
                                                      const int32_t* __restrict__ sl_rows,
                                                      const int64_t* __restrict__ off,
                                                      const int32_t* __restrict__ ell_col,
                                                      const double* __restrict__ ell_val, int32_t c,
                                                      AT* __restrict__ out) {
  const int sl = blockIdx.x, l = threadIdx.x;
  const int64_t o0 = off[sl];
  const int w = (int)((off[sl + 1] - o0) / 64);
  const bool live = l < sl_rows[sl];
  const int64_t row = sl_row[sl] + l;
  for (int q = 0; q < w; ++q) {
    double v = 0.0;
    if (live && ell_col[row * c + q] >= 0) v = ell_val[row * c + q];
    out[o0 + 64 * q + l] = (AT)v;
  }
}

// ---------------------------------------------------------------------------
// Dense SPD inverses (coarse blocks and local levels): Gauss-Jordan on blocks
// of at most kCNB rows, recursive Schur complements above.

constexpr int kCNB = 64;

constexpr int kPivThreads = 256;

// Gauss-Jordan inverse of a w x w (w <= 64) block held in registers: thread x
// owns the 4 x 4 sub-block at rows 4 (x / 16).., columns 4 (x % 16)..; each
// step publishes only the pivot row and column through LDS (double-buffered,
// one barrier per step).  On return m holds the inverse (identity outside w x w).
__device__ inline void gj_regs(double (&m)[4][4], int w, int32_t* err, int sub, int blk, int row0) {
  __shared__ double prow[2][kCNB], pcol[2][kCNB];
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;  // this thread's 4 x 4 block
  const int r0 = tr * 4, c0 = tc * 4;
  // rows and columns past w become identity (zero outside the diagonal on entry), so
  // the pivots run in groups of four whose position inside a block is known at
  // compile time; identity rows keep pivot 1 and leave the others untouched
  if (tr == tc) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (r0 + i >= w) m[i][i] = 1.0;
  }
  const int nq = (w + 3) >> 2;
  for (int tau = 0; tau < nq; ++tau) {
    const bool prow_mine = tr == tau, pcol_mine = tc == tau;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = 4 * tau + u;
      const int buf = u & 1;
      if (prow_mine)
#pragma unroll
        for (int j = 0; j < 4; ++j) prow[buf][c0 + j] = m[u][j];
      if (pcol_mine)
#pragma unroll
        for (int i = 0; i < 4; ++i) pcol[buf][r0 + i] = m[i][u];
      __syncthreads();
      double d = prow[buf][t];
      if (t < w && (!(d > 0.0) || !isfinite(d))) {
        if (threadIdx.x == 0) record_error(err, DDG_ERR_NOT_SPD, sub, blk, row0 + t);
        d = 1.0;
      }
      const double rd = 1.0 / d;
      // branch-free step: with P_i = rd on the pivot row (else -a_it rd) and Q_j = 1 on
      // the pivot column (else a_tj), every entry becomes (row t or column t ? 0 : a_ij)
      // + P_i Q_j
      double P[4], Q[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) P[i] = (prow_mine && i == u) ? rd : -pcol[buf][r0 + i] * rd;
#pragma unroll
      for (int j = 0; j < 4; ++j) Q[j] = (pcol_mine && j == u) ? 1.0 : prow[buf][c0 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool zero = (prow_mine && i == u) || (pcol_mine && j == u);
          m[i][j] = __builtin_fma(P[i], Q[j], zero ? 0.0 : m[i][j]);
        }
      // a buffer is rewritten two steps later, after the next step's barrier
    }
  }
}

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Recursive inverse of one dense SPD block (the coarse matrix of a single
// system).  With A = [[A11, A12], [A21, A22]], W = A11^{-1} A12 and the Schur
// complement S = A22 - A21 W:
//   A^{-1} = [[A11^{-1} + W S^{-1} W^T, -W S^{-1}], [-S^{-1} W^T, S^{-1}]],
// so the work is two half-size inverses and four GEMMs; the GEMMs run on the
// FP64 matrix cores and carry almost all of the N^3 flops, which keeps the
// inversion compute-bound instead of making N/64 passes over the matrix.
// Leaves (at most 64 rows) are inverted by Gauss-Jordan in LDS.

struct GemmArgs {
  const double* A;  // M x K, row-major, lda
  int64_t lda;
  const double* B;  // K x N row-major (ldb), or N x K row-major when tb
  int64_t ldb;
  int32_t tb;
  double* C;        // M x N, row-major, ldc
  int64_t ldc;
  int32_t M, N, K;
  double alpha, beta;
  // epilogue: 0 plain; 1 symmetric result (M = N): the tile's entries on and below the
  // diagonal are formed and the ones below it also written to their mirror, so C
  // comes out exactly symmetric (the caller runs only tiles with i0 >= j0); 2 also
  // writes the transpose into D (ldd)
  int32_t mode;
  double* D;
  int64_t ldd;
};

// C = beta C + alpha A op(B) on 64 x 64 output tiles on the FP64 matrix cores: each of
// the 4 waves computes a 32 x 32 quadrant as 2 x 2 products of 16 x 16 tiles
// (v_mfma_f64_16x16x4: lane l feeds A[l%16][l/16] and B[l/16][l%16] and receives
// D[4r + l/16][l%16] in result register r), the operands staged through LDS in
// 32-wide chunks of the reduction dimension.  The next chunk's global loads are
// issued into registers before the current chunk's products, so their latency
// overlaps the matrix-core work.
__device__ inline void gemm_tile(const GemmArgs& g, int64_t i0, int64_t j0) {
  constexpr int UC = 32;
  constexpr int PER = 64 * UC / 256;  // elements of each operand chunk per thread
  // the operand chunks, and after the reduction the output tile for the mirrored or
  // transposed stores
  __shared__ double smem[64 * (UC + 1) + UC * (64 + 1)];
  double (*As)[UC + 1] = reinterpret_cast<double (*)[UC + 1]>(smem);
  double (*Bs)[64 + 1] = reinterpret_cast<double (*)[64 + 1]>(smem + 64 * (UC + 1));
  double (*Cs)[64 + 1] = reinterpret_cast<double (*)[64 + 1]>(smem);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  mfma_d4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  double ra[PER], rb[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * 256;
      const int r = idx / UC, u = idx % UC;
      ra[q] = (i0 + r < g.M && k0 + u < g.K) ? g.A[(i0 + r) * g.lda + k0 + u] : 0.0;
      if (g.tb) {
        rb[q] = (j0 + r < g.N && k0 + u < g.K) ? g.B[(j0 + r) * g.ldb + k0 + u] : 0.0;
      } else {
        const int uu = idx / 64, c = idx % 64;
        rb[q] = (j0 + c < g.N && k0 + uu < g.K) ? g.B[(int64_t)(k0 + uu) * g.ldb + j0 + c] : 0.0;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int idx = threadIdx.x + q * 256;
      const int r = idx / UC, u = idx % UC;
      As[r][u] = ra[q];
      if (g.tb) Bs[u][r] = rb[q];
      else Bs[idx / 64][idx % 64] = rb[q];
    }
  };
  fetch(0);
  stash();
  __syncthreads();
  for (int k0 = 0; k0 < g.K; k0 += UC) {
    const bool more = k0 + UC < g.K;
    if (more) fetch(k0 + UC);
#pragma unroll
    for (int kk = 0; kk < UC; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) af[x] = As[wr + x * 16 + li][kk + lk];
#pragma unroll
      for (int y = 0; y < 2; ++y) bf[y] = Bs[kk + lk][wc + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stash();
      __syncthreads();
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int li_ = wr + x * 16 + 4 * r + lk, lj_ = wc + y * 16 + li;
        const int64_t i = i0 + li_;
        const int64_t j = j0 + lj_;
        if (i >= g.M || j >= g.N || (g.mode == 1 && j > i)) continue;
        double* c = g.C + i * g.ldc + j;
        const double v = (g.beta == 0.0 ? 0.0 : g.beta * *c) + g.alpha * acc[x][y][r];
        *c = v;
        if (g.mode != 0) Cs[li_][lj_] = v;
      }
  if (g.mode == 0) return;
  // mirrored (mode 1: C[j][i], below the diagonal only) or transposed (mode 2:
  // D[j][i]) stores, rows of the stored matrix along the threads
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int lj_ = idx >> 6, li_ = idx & 63;
    const int64_t i = i0 + li_, j = j0 + lj_;
    if (i >= g.M || j >= g.N) continue;
    if (g.mode == 1) {
      if (i > j) g.C[j * g.ldc + i] = Cs[li_][lj_];
    } else {
      g.D[j * g.ldd + i] = Cs[li_][lj_];
    }
  }
}

// tile t of the packed inverses (system tile_inst[t]); zero beyond the block's order
__global__ void k_pack_coarse(const double* __restrict__ A, const int64_t* __restrict__ a0_off,
                              const int32_t* __restrict__ nblk, const int32_t* __restrict__ tile_inst,
                              const int64_t* __restrict__ tile_base, int64_t ntiles, double* __restrict__ out) {
  constexpr int T = 64;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * T * T) return;
  const int64_t t = idx / (T * T);
  const int sys = tile_inst[t];
  const int64_t N = nblk[sys];
  const double* Ab = A + a0_off[sys];
  int rr, cc;
  tile_rc<double, T>((int)(idx % (T * T)), rr, cc);
  int I, J;
  tile_ij((int)(t - tile_base[sys]), I, J);
  const int64_t row = (int64_t)I * T + rr;
  const int64_t col = (int64_t)J * T + cc;
  double v = 0.0;
  if (row < N && col < N) v = (row >= col) ? Ab[row * N + col] : Ab[col * N + row];
  out[idx] = v;
}

// Batched recursive inverse of the level matrices of one stage (item q: S at
// scratch + off[q], n[q] x n[q], leading dimension n[q]).  The recursion tree is
// built on the stage's widest level; an item takes each node [lo, hi) with split
// m clipped to its own size, so one launch per node serves every item.
struct BInv {
  double* scratch;
  const int64_t* off;
  const int32_t* n;
  double* W;          // per item workspace: wstride elements each, or at woffs[q] when given
  int64_t wstride;
  const int64_t* woffs;
  const int32_t* err_sub;   // NULL: a coarse block (reported as coarse row)
  const int32_t* err_blk;
};

__device__ inline double* binv_work(const BInv& bi, int q) {
  return bi.W + (bi.woffs ? bi.woffs[q] : (int64_t)q * bi.wstride);
}

__global__ void __launch_bounds__(kPivThreads) k_bleaf(BInv bi, int lo, int hi, int32_t* err) {
  const int q = blockIdx.x;
  const int b = bi.n[q];
  if (lo >= b) return;
  const int w = min(hi, b) - lo;
  double* X = bi.scratch + bi.off[q] + (int64_t)lo * b + lo;
  const int r0 = (threadIdx.x >> 4) * 4, c0 = (threadIdx.x & 15) * 4;
  double m[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) m[i][j] = (r0 + i < w && c0 + j < w) ? X[(int64_t)(r0 + i) * b + c0 + j] : 0.0;
  if (bi.err_sub) gj_regs(m, w, err, bi.err_sub[q], bi.err_blk[q], lo);
  else gj_regs(m, w, err, -1, bi.err_blk ? bi.err_blk[q] : q, lo);
  // the inverse made exactly symmetric, (X + X^T) / 2 with the entry below the
  // diagonal first, through LDS
  __shared__ double sm[64][65];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) sm[r0 + i][c0 + j] = m[i][j];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + i, c = c0 + j;
      if (r >= w || c >= w) continue;
      const double v = r > c ? 0.5 * (sm[r][c] + sm[c][r]) : r < c ? 0.5 * (sm[c][r] + sm[r][c]) : sm[r][r];
      X[(int64_t)r * b + c] = v;
    }
}

// op 0: W = X11 X12; 1: X22 -= X21 W (the Schur complement, formed on and below the
// diagonal and mirrored); 2: X12 = -W X22, with X21 = X12^T; 3: X11 -= X12 W^T
// (formed on and below the diagonal and mirrored).
// The occupancy hint makes the compiler keep the accumulators in VGPRs: 154 in all
// instead of 160 VGPRs + 32 AGPRs, so three waves per SIMD fit where two did, and the
// operand loads of more tiles overlap (the products are the same instructions).
__global__ void __launch_bounds__(256, 2) k_bgemm(BInv bi, int op, int lo, int mid, int hi, int64_t woff, int ldw) {
  const int q = blockIdx.z;
  const int b = bi.n[q];
  if (lo >= b) return;
  const int m = min(mid, b), h = min(hi, b);
  const int n1 = m - lo, n2 = h - m;
  if (n2 <= 0) return;
  double* X = bi.scratch + bi.off[q];
  double* W = binv_work(bi, q) + woff;
  double* X11 = X + (int64_t)lo * b + lo;
  double* X12 = X + (int64_t)lo * b + m;
  double* X21 = X + (int64_t)m * b + lo;
  double* X22 = X + (int64_t)m * b + m;
  GemmArgs g;
  switch (op) {
    case 0: g = GemmArgs{X11, b, X12, b, 0, W, ldw, n1, n2, n1, 1.0, 0.0, 0, nullptr, 0}; break;
    case 1: g = GemmArgs{X21, b, W, ldw, 0, X22, b, n2, n2, n1, -1.0, 1.0, 1, nullptr, 0}; break;
    case 2: g = GemmArgs{W, ldw, X22, b, 0, X12, b, n1, n2, n2, -1.0, 0.0, 2, X21, b}; break;
    default: g = GemmArgs{X12, b, W, ldw, 1, X11, b, n1, n1, n2, -1.0, 1.0, 1, nullptr, 0}; break;
  }
  const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
  if (i0 >= g.M || j0 >= g.N) return;
  if (g.mode == 1 && j0 > i0) return;   // symmetric results: lower tiles only
  gemm_tile(g, i0, j0);
}

// Symmetry.  The recursive inverse forms the Schur complement D - C W and the update
// X11 - X12 W^T, whose two triangles would differ by rounding, and Gauss-Jordan
// leaves are not exactly symmetric either.  Used as they are in the next step, that
// asymmetry grows from node to node and from level to level when the operator is
// ill-conditioned or the level couplings amplify (||X C|| > 1: the 13-point
// biharmonic operator).  So every leaf is made exactly symmetric ((X + X^T) / 2,
// in k_bleaf), and the two symmetric updates are formed on and below the diagonal
// only and mirrored (k_bgemm ops 1 and 3).

// Workspace elements per item that binv_node(lo = 0, hi = n) touches: W of a node
// sits at the node's stack offset and spans n1 x n2 (leading dimension n2).
int64_t binv_work_need(int lo, int hi, int64_t woff) {
  const int n = hi - lo;
  if (n <= kCNB) return woff;
  const int m = lo + kCNB * ((n + 2 * kCNB - 1) / (2 * kCNB));
  const int64_t next = woff + (int64_t)(m - lo) * (hi - m);
  return std::max(next, std::max(binv_work_need(lo, m, next), binv_work_need(m, hi, next)));
}

// Inverse of X[lo:hi, lo:hi] in place (the items' blocks past their order are
// skipped), symmetric on return.
void binv_node(hipStream_t s, const BInv& bi, unsigned cnt, int lo, int hi, int64_t woff, int32_t* err) {
  const int n = hi - lo;
  if (n <= kCNB) {
    hipLaunchKernelGGL(k_bleaf, dim3(cnt), dim3(kPivThreads), 0, s, bi, lo, hi, err);
    return;
  }
  const int m = lo + kCNB * ((n + 2 * kCNB - 1) / (2 * kCNB));
  const int n1 = m - lo, n2 = hi - m;
  const int64_t next = woff + (int64_t)n1 * n2;
  auto gemm_grid = [&](int M, int N) { return dim3((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), cnt); };
  binv_node(s, bi, cnt, lo, m, next, err);
  hipLaunchKernelGGL(k_bgemm, gemm_grid(n1, n2), dim3(256), 0, s, bi, 0, lo, m, hi, woff, n2);
  hipLaunchKernelGGL(k_bgemm, gemm_grid(n2, n2), dim3(256), 0, s, bi, 1, lo, m, hi, woff, n2);
  binv_node(s, bi, cnt, m, hi, next, err);
  hipLaunchKernelGGL(k_bgemm, gemm_grid(n1, n2), dim3(256), 0, s, bi, 2, lo, m, hi, woff, n2);
  hipLaunchKernelGGL(k_bgemm, gemm_grid(n1, n1), dim3(256), 0, s, bi, 3, lo, m, hi, woff, n2);
}

// Schedule of the batched factorisation: groups of subdomains whose scratch
// fits the budget; per group, the chain steps, then the middle level.
struct FacPlanHost {
  struct Stage {
    int32_t first, count;    // items [first, first + count) of the item array
    int32_t gj;              // 1: invert and pack after forming (0: a form-only pass)
    int32_t bmax;            // widest level of the stage
  };
  std::vector<FacItem> items;
  std::vector<Stage> stages;
  std::vector<int32_t> group_first;   // stage index where each group starts
  int64_t scratch_elems = 0, tm_elems = 0;
  int32_t max_items = 0;
};

void build_fac_plan(const Symbolic& S, FacPlanHost& P) {
  const int64_t bmax = std::max<int32_t>(1, S.max_blk);
  const int64_t per_chain = 2 * bmax * bmax;            // X and S buffers
  const int64_t budget = ((int64_t)5 << 30) / 8;        // scratch elements (+ Tm of the same order)
  // (at most 30000 subdomains per group: item counts stay within a grid dimension)
  const int32_t gsub = (int32_t)std::max<int64_t>(
      1, std::min<int64_t>(std::min<int64_t>(S.n_parts, 30000), budget / (2 * per_chain)));
  P.scratch_elems = (int64_t)gsub * 2 * per_chain;
  P.tm_elems = (int64_t)gsub * 2 * bmax * bmax;
  for (int32_t g0 = 0; g0 < S.n_parts; g0 += gsub) {
    const int32_t g1 = std::min(S.n_parts, g0 + gsub);
    P.group_first.push_back((int32_t)P.stages.size());
    int32_t steps = 0;
    for (int32_t i = g0; i < g1; ++i) {
      const int32_t K = S.sub_blk_ptr[i + 1] - S.sub_blk_ptr[i];
      const int32_t m = S.sub_mid[i];
      steps = std::max(steps, std::max(m, K - 1 - m));
    }
    // chain (i, dir) uses buffers at ((i - g0) * 2 + dir) * per_chain + {0, bmax^2}; after
    // step j its inverse sits in buffer j & 1
    auto buf = [&](int32_t i, int dir, int par) {
      return ((int64_t)(i - g0) * 2 + dir) * per_chain + (par & 1) * bmax * bmax;
    };
    for (int32_t j = 0; j < steps; ++j) {
      FacPlanHost::Stage st{(int32_t)P.items.size(), 0, 1, 0};
      for (int32_t i = g0; i < g1; ++i) {
        const int32_t kb0 = S.sub_blk_ptr[i], K = S.sub_blk_ptr[i + 1] - kb0;
        const int32_t m = S.sub_mid[i], nB = K - 1 - m;
        for (int dir = 0; dir < 2; ++dir) {
          const int32_t len = dir == 0 ? m : nB;
          if (j >= len) continue;
          const int32_t k = dir == 0 ? j : K - 1 - j;
          const int32_t kp = dir == 0 ? k - 1 : k + 1;
          FacItem it{};
          it.cur = kb0 + k;
          it.prev = j > 0 ? kb0 + kp : -1;
          it.sub = i;
          it.use_up = dir;
          it.add_d = 1;
          it.s_off = buf(i, dir, j);
          it.x_off = buf(i, dir, j - 1);
          it.t_off = (int64_t)(P.items.size() - st.first) * bmax * bmax;
          st.bmax = std::max(st.bmax, S.blk_size[it.cur]);
          P.items.push_back(it);
        }
      }
      st.count = (int32_t)P.items.size() - st.first;
      if (st.count) P.stages.push_back(st);
    }
    // middle level: formed in the top chain's free buffer from both chains' last inverses
    for (int pass = 0; pass < 2; ++pass) {
      FacPlanHost::Stage st{(int32_t)P.items.size(), 0, pass == 1, 0};
      for (int32_t i = g0; i < g1; ++i) {
        const int32_t kb0 = S.sub_blk_ptr[i], K = S.sub_blk_ptr[i + 1] - kb0;
        const int32_t m = S.sub_mid[i], nB = K - 1 - m;
        FacItem it{};
        it.cur = kb0 + m;
        it.sub = i;
        it.s_off = buf(i, 0, m);
        it.t_off = (int64_t)(P.items.size() - st.first) * bmax * bmax;
        if (pass == 0) {
          it.prev = m > 0 ? kb0 + m - 1 : -1;
          it.use_up = 0;
          it.add_d = 1;
          it.x_off = buf(i, 0, m - 1);
        } else {
          it.prev = nB > 0 ? kb0 + m + 1 : -1;
          it.use_up = 1;
          it.add_d = 0;
          it.x_off = buf(i, 1, nB - 1);
        }
        st.bmax = std::max(st.bmax, S.blk_size[it.cur]);
        P.items.push_back(it);
      }
      st.count = (int32_t)P.items.size() - st.first;
      P.stages.push_back(st);
    }
  }
  for (auto& st : P.stages) P.max_items = std::max(P.max_items, st.count);
}

template <class FT, int T>
void launch_factor_t(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  if (!h.fac_plan_ready) {
    FacPlanHost P;
    build_fac_plan(S, P);
    h.fac_items.upload(P.items, s);
    h.fac_stages.clear();
    for (auto& st : P.stages) h.fac_stages.push_back({st.first, st.count, st.gj, st.bmax});
    // per-item arrays of the inversion kernels, one block per stage (same item order)
    std::vector<int64_t> off(P.items.size());
    std::vector<int32_t> n(P.items.size()), esub(P.items.size()), eblk(P.items.size());
    const int64_t bmax = std::max<int32_t>(1, S.max_blk);
    for (auto& st : P.stages)
      for (int32_t q = 0; q < st.count; ++q) {
        const FacItem& it = P.items[st.first + q];
        off[st.first + q] = it.s_off;
        n[st.first + q] = S.blk_size[it.cur];
        esub[st.first + q] = it.sub;
        eblk[st.first + q] = it.cur - S.sub_blk_ptr[it.sub];
      }
    h.fac_off.upload(off, s);
    h.fac_n.upload(n, s);
    h.fac_esub.upload(esub, s);
    h.fac_eblk.upload(eblk, s);
    h.fac_scratch.alloc((size_t)P.scratch_elems * sizeof(double));
    h.fac_tm.alloc((size_t)P.tm_elems * sizeof(double));
    h.fac_wstride = binv_work_need(0, (int)bmax, 0) + 64;
    h.fac_work.alloc((size_t)h.fac_wstride * P.max_items * sizeof(double));
    h.fac_max_items = P.max_items;
    h.fac_plan_ready = true;
  }
  FacArgs a;
  a.set_ptr = h.set_ptr.as<int64_t>();
  a.sub_blk_ptr = h.sub_blk_ptr.as<int32_t>();
  a.blk_start = h.blk_start.as<int32_t>();
  a.blk_size = h.blk_size.as<int32_t>();
  a.blk_foff = h.blk_foff.as<int64_t>();
  a.lo_col = h.lo_col.as<int32_t>();
  a.lo_val = h.lo_val.as<double>();
  a.cl = S.cl;
  a.up_col = h.up_col.as<int32_t>();
  a.up_val = h.up_val.as<double>();
  a.cu = S.cu;
  a.in_ptr = h.in_ptr.as<int64_t>();
  a.in_col = h.in_col.as<int32_t>();
  a.in_pos = h.in_pos.as<int64_t>();
  a.val = h.val.as<double>();
  a.scratch = h.fac_scratch.as<double>();
  a.tm = h.fac_tm.as<double>();
  a.fac = h.fac.p;
  const FacItem* items = h.fac_items.as<FacItem>();
  for (const auto& st : h.fac_stages) {
    a.items = items + st.first;
    const unsigned ny = (unsigned)((st.bmax + kFacRows - 1) / kFacRows);
    hipLaunchKernelGGL(k_fac_tm, dim3((unsigned)st.count, ny), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_fac_form, dim3((unsigned)st.count, ny), dim3(256), 0, s, a);
    if (!st.gj) continue;
    BInv bi;
    bi.scratch = a.scratch;
    bi.off = h.fac_off.as<int64_t>() + st.first;
    bi.n = h.fac_n.as<int32_t>() + st.first;
    bi.W = h.fac_work.as<double>();
    bi.wstride = h.fac_wstride;
    bi.woffs = nullptr;
    bi.err_sub = h.fac_esub.as<int32_t>() + st.first;
    bi.err_blk = h.fac_eblk.as<int32_t>() + st.first;
    const unsigned cnt = (unsigned)st.count;
    binv_node(s, bi, cnt, 0, st.bmax, 0, h.err_flag.as<int32_t>());
    const int64_t nt = (st.bmax + T - 1) / T;
    const unsigned py = (unsigned)std::min<int64_t>(64, (nt * (nt + 1) / 2 * T * T + 255) / 256);
    hipLaunchKernelGGL((k_fac_pack<FT, T>), dim3(cnt, py), dim3(256), 0, s, a);
  }
  DDG_HIP(hipGetLastError());
}

template <class FT>
void launch_factor_p(Handle& h, hipStream_t s) {
  switch (h.S.tile) {
    case 16: launch_factor_t<FT, 16>(h, s); break;
    case 32: launch_factor_t<FT, 32>(h, s); break;
    default: launch_factor_t<FT, 64>(h, s); break;
  }
}

}  // namespace

void launch_coarse_basis(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  DDG_REQUIRE(h.k <= kMaxGen, DDG_ERR_UNSUPPORTED, "at most 80 generating vectors");
  DevBuf work;
  work.alloc((size_t)S.n * h.k * sizeof(double));
  auto kern = h.k <= 32 ? k_coarse_qr<32> : k_coarse_qr<kMaxGen>;
  hipLaunchKernelGGL(kern, dim3(S.n_parts), dim3(kQrThreads), 0, s, h.own_ptr.as<int64_t>(),
                     h.own_idx.as<int32_t>(), h.F.as<double>(), S.n, h.k, h.opt.rank_tol,
                     work.as<double>(), h.Q.as<double>(), h.kcnt_d.as<int32_t>(), h.err_flag.as<int32_t>());
  DDG_HIP(hipGetLastError());
  DDG_HIP(hipStreamSynchronize(s));
}

void launch_galerkin(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  DDG_HIP(hipMemsetAsync(h.A0.p, 0, (size_t)h.a0_off[h.nb] * sizeof(double), s));
  auto kern = h.k <= 32 ? k_galerkin<2, 4> : k_galerkin<5, 2>;
  hipLaunchKernelGGL(kern, dim3(S.n_parts), dim3(kGalThreads), 0, s, h.own_ptr.as<int64_t>(),
                     h.own_idx.as<int32_t>(), h.nbr_ptr.as<int32_t>(), h.nbr_idx.as<int32_t>(),
                     h.part.as<int32_t>(), h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(),
                     h.Q.as<double>(), h.k, h.rowptr.as<int64_t>(), h.col.as<int32_t>(),
                     h.val.as<double>(), h.sub_inst.as<int32_t>(), h.cblk_off_d.as<int64_t>(),
                     h.cblk_n_d.as<int32_t>(), h.a0_off_d.as<int64_t>(), h.A0.as<double>());
  DDG_HIP(hipGetLastError());
}

void launch_coarse_invert(Handle& h, hipStream_t s) {
  const int64_t total = h.a0_off[h.nb];
  // the inverse is formed in a copy so that A0 stays available for export; the
  // buffers stay with the handle (freeing device memory would synchronise the device)
  DevBuf& inv = h.cinv;
  if (inv.bytes < (size_t)total * sizeof(double)) inv.alloc((size_t)total * sizeof(double));
  DDG_HIP(hipMemcpyAsync(inv.p, h.A0.p, (size_t)total * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (h.cinv_groups.empty()) {
    // recursive inverse of every coarse block, one item per system: systems sorted by
    // order and taken in groups whose workspace (the tree of the group's largest
    // block, for every item) stays within a budget.  The group tables depend only on
    // the structure: built and uploaded once per handle, so a refactor enqueues the
    // whole inverse without waiting on the host.
    int64_t nmax = 0;
    for (int32_t b = 0; b < h.nb; ++b) nmax = std::max<int64_t>(nmax, h.cblk_n[b]);
    std::vector<int32_t> order(h.nb);
    for (int32_t b = 0; b < h.nb; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return h.cblk_n[x] > h.cblk_n[y]; });
    const int64_t budget = ((int64_t)1 << 30) / 8;   // workspace elements (1 GiB)
    const int64_t need0 = binv_work_need(0, (int)nmax, 0) + 64;
    const size_t wbytes = (size_t)std::max(need0, std::min<int64_t>(budget, need0 * h.nb)) * sizeof(double);
    if (h.cwork.bytes < wbytes) h.cwork.alloc(wbytes);
    std::vector<int64_t> goff;
    std::vector<int32_t> gn, gsys;
    for (int32_t i0 = 0; i0 < h.nb;) {
      const int32_t nfirst = h.cblk_n[order[i0]];
      if (nfirst == 0) break;   // the remaining systems have no coarse space
      const int64_t need = binv_work_need(0, nfirst, 0) + 64;
      const int32_t cnt =
          (int32_t)std::max<int64_t>(1, std::min<int64_t>(h.nb - i0, (int64_t)(h.cwork.bytes / 8) / need));
      h.cinv_groups.push_back(Handle::CoarseGroup{i0, cnt, nfirst, need});
      for (int32_t q = 0; q < cnt; ++q) {
        goff.push_back(h.a0_off[order[i0 + q]]);
        gn.push_back(h.cblk_n[order[i0 + q]]);
        gsys.push_back(order[i0 + q]);
      }
      i0 += cnt;
    }
    const size_t m = goff.size();
    h.cgd.alloc(std::max<size_t>(1, m) * (sizeof(int64_t) + 2 * sizeof(int32_t)));
    if (m) {
      int64_t* doff = h.cgd.as<int64_t>();
      int32_t* dn = reinterpret_cast<int32_t*>(doff + m);
      DDG_HIP(hipMemcpyAsync(doff, goff.data(), m * sizeof(int64_t), hipMemcpyHostToDevice, s));
      DDG_HIP(hipMemcpyAsync(dn, gn.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
      DDG_HIP(hipMemcpyAsync(dn + m, gsys.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
      // (pageable sources: wait for the copies before the vectors go out of scope)
      DDG_HIP(hipStreamSynchronize(s));
    }
    h.cinv_items = (int32_t)m;
  }
  const int64_t m = h.cinv_items;
  int64_t* doff = h.cgd.as<int64_t>();
  int32_t* dn = reinterpret_cast<int32_t*>(doff + m);
  int32_t* dsys = dn + m;
  for (const auto& gr : h.cinv_groups) {
    BInv bi;
    bi.scratch = inv.as<double>();
    bi.off = doff + gr.first;
    bi.n = dn + gr.first;
    bi.W = h.cwork.as<double>();
    bi.wstride = gr.need;
    bi.woffs = nullptr;
    bi.err_sub = nullptr;
    bi.err_blk = dsys + gr.first;
    binv_node(s, bi, (unsigned)gr.count, 0, gr.nfirst, 0, h.err_flag.as<int32_t>());
  }
  const int64_t elems = h.ntiles * 64 * 64;
  hipLaunchKernelGGL(k_pack_coarse, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, inv.as<double>(),
                     h.a0_off_d.as<int64_t>(), h.cblk_n_d.as<int32_t>(), h.tile_inst.as<int32_t>(),
                     h.tile_base_d.as<int64_t>(), h.ntiles, h.A0inv_t.as<double>());
  DDG_HIP(hipGetLastError());
}

void launch_local_factor(Handle& h, hipStream_t s) {
  switch (h.opt.precision) {
    case DDG_MIXED_FP32: launch_factor_p<float>(h, s); break;
    case DDG_MIXED_BF16: launch_factor_p<__hip_bfloat16>(h, s); break;
    default: launch_factor_p<double>(h, s); break;
  }
}

template <class AT>
void refresh_sliced(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  const int32_t nsl = (int32_t)S.sl_rows.size();
  if (nsl == 0) return;
  hipLaunchKernelGGL(k_gather_sliced<AT>, dim3((unsigned)nsl), dim3(64), 0, s, h.sl_row.as<int64_t>(),
                     h.sl_rows.as<int32_t>(), h.sl_lo_off.as<int64_t>(), h.lo_col.as<int32_t>(),
                     h.lo_val.as<double>(), S.cl, h.sl_lo_val.as<AT>());
  hipLaunchKernelGGL(k_gather_sliced<AT>, dim3((unsigned)nsl), dim3(64), 0, s, h.sl_row.as<int64_t>(),
                     h.sl_rows.as<int32_t>(), h.sl_up_off.as<int64_t>(), h.up_col.as<int32_t>(),
                     h.up_val.as<double>(), S.cu, h.sl_up_val.as<AT>());
}

void launch_gather(const int64_t* pos, const double* src, double* dst, int64_t m, hipStream_t s) {
  if (m == 0) return;
  hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, pos, src, dst, m);
  DDG_HIP(hipGetLastError());
}

void launch_refresh_couplings(Handle& h, hipStream_t s) {
  const int64_t nlo = (int64_t)h.S.lo_pos.size(), nup = (int64_t)h.S.up_pos.size();
  if (nlo)
    hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((nlo + 255) / 256)), dim3(256), 0, s,
                       h.lo_pos.as<int64_t>(), h.val.as<double>(), h.lo_val.as<double>(), nlo);
  if (nup)
    hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, s,
                       h.up_pos.as<int64_t>(), h.val.as<double>(), h.up_val.as<double>(), nup);
  if (h.S.sliced) {
    if (h.opt.precision == DDG_FP64) refresh_sliced<double>(h, s);
    else refresh_sliced<float>(h, s);
  }
  DDG_HIP(hipGetLastError());
}

}  // namespace ddg
