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

constexpr int kMaxKq = 32;

// Error record: [0] = code (0 none), [1] = subdomain, [2] = block, [3] = local row
__device__ inline void record_error(int32_t* err, int code, int sub, int blk, int row) {
  if (atomicCAS(err, 0, code) == 0) {
    err[1] = sub;
    err[2] = blk;
    err[3] = row;
  }
}

// Sum `cnt` per-thread values across a 256-thread workgroup; results in out[0..cnt).
template <int NT>
__device__ inline void multi_sum(double (&acc)[kMaxKq], int cnt, double* red /*[NT/64][kMaxKq]*/,
                                 double* out) {
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < kMaxKq; ++m) {
    if (m < cnt) {
      double v = wave_sum(acc[m]);
      if ((threadIdx.x & 63) == 0) red[wv * kMaxKq + m] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) s += red[w * kMaxKq + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Coarse basis

constexpr int kQrThreads = 256;

__global__ void __launch_bounds__(kQrThreads) k_coarse_qr(
    const int64_t* __restrict__ own_ptr, const int32_t* __restrict__ own_idx,
    const double* __restrict__ F, int64_t n, int k, double rank_tol, double* __restrict__ work,
    double* __restrict__ Q, int32_t* __restrict__ kcnt, int32_t* __restrict__ err) {
  __shared__ double red[(kQrThreads / 64) * kMaxKq];
  __shared__ double sums[kMaxKq];
  __shared__ int used[kMaxKq];
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
  if (tid < kMaxKq) used[tid] = 0;
  __syncthreads();
  int kept = 0;
  double acc[kMaxKq];
  for (int s = 0; s < k; ++s) {
    // residual norms of the unused columns
#pragma unroll
    for (int m = 0; m < kMaxKq; ++m) acc[m] = 0.0;
    for (int r = tid; r < ni; r += kQrThreads) {
#pragma unroll
      for (int m = 0; m < kMaxKq; ++m)
        if (m < k) {
          double v = V[(int64_t)m * ni + r];
          acc[m] += v * v;
        }
    }
    multi_sum<kQrThreads>(acc, k, red, sums);
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
      for (int m = 0; m < kMaxKq; ++m) acc[m] = 0.0;
      for (int r = tid; r < ni; r += kQrThreads) {
        const int g = own_idx[base + r];
        const double v = vp[r];
#pragma unroll
        for (int m = 0; m < kMaxKq; ++m)
          if (m < kept) acc[m] += Q[(int64_t)g * k + m] * v;
      }
      multi_sum<kQrThreads>(acc, kept, red, sums);
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
    multi_sum<kQrThreads>(acc, 1, red, sums);
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
    for (int m = 0; m < kMaxKq; ++m) acc[m] = 0.0;
    for (int r = tid; r < ni; r += kQrThreads) {
      const double qv = vp[r];
#pragma unroll
      for (int m = 0; m < kMaxKq; ++m)
        if (m < k && m != jp && !used[m]) acc[m] += qv * V[(int64_t)m * ni + r];
    }
    multi_sum<kQrThreads>(acc, k, red, sums);
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
constexpr int kGalAcc = 16;
constexpr int kGalLds = 48 * 1024;

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
  const int tid = threadIdx.x;
  // slots per group so that every thread holds at most kGalAcc accumulators
  const int per_slot = kq * kq;
  int gslots = (kGalThreads * kGalAcc) / per_slot;
  if (gslots < 1) gslots = 1;
  for (int g0 = 0; g0 < nnb; g0 += gslots) {
    const int gs = min(gslots, nnb - g0);
    const int entries = gs * per_slot;
    int ch = kGalLds / (8 * (gs * kq + kq));
    if (ch > 64) ch = 64;
    double* Wc = lds;               // [ch][gs][kq]
    double* Qc = lds + ch * gs * kq;  // [ch][kq]
    double acc[kGalAcc];
#pragma unroll
    for (int u = 0; u < kGalAcc; ++u) acc[u] = 0.0;
    for (int r0 = 0; r0 < ni; r0 += ch) {
      const int rows = min(ch, ni - r0);
      for (int idx = tid; idx < rows * gs * kq; idx += kGalThreads) {
        const int r = idx / (gs * kq);
        const int s = (idx / kq) % gs;
        const int b = idx % kq;
        const int g = own_idx[base + r0 + r];
        const int j = nbr_idx[nb0 + g0 + s];
        double w = 0.0;
        for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
          const int c = ci[t];
          if (part[c] == j) w += val[t] * Q[(int64_t)c * kq + b];
        }
        Wc[idx] = w;
      }
      for (int idx = tid; idx < rows * kq; idx += kGalThreads) {
        const int r = idx / kq, a = idx % kq;
        Qc[idx] = Q[(int64_t)own_idx[base + r0 + r] * kq + a];
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kGalAcc; ++u) {
        const int e = tid + u * kGalThreads;
        if (e < entries) {
          const int s = e / per_slot;
          const int a = (e / kq) % kq;
          const int b = e % kq;
          double v = acc[u];
          for (int r = 0; r < rows; ++r) v += Qc[r * kq + a] * Wc[(r * gs + s) * kq + b];
          acc[u] = v;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kGalAcc; ++u) {
      const int e = tid + u * kGalThreads;
      if (e < entries) {
        const int s = e / per_slot;
        const int a = (e / kq) % kq;
        const int b = e % kq;
        const int j = nbr_idx[nb0 + g0 + s];
        if (a < ki && b < kcnt[j]) A0b[(koff[i] + a - c0) * nc + koff[j] + b - c0] = acc[u];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// In-workgroup helpers for Gauss-Jordan inversion of a small SPD block in LDS.
// piv is w x w with leading dimension ldp; on return it holds the inverse.
template <int NT>
__device__ inline void gj_small(double* piv, int w, int ldp, int32_t* err, int sub, int blk, int row0) {
  for (int t = 0; t < w; ++t) {
    double d = piv[t * ldp + t];
    const bool bad = !(d > 0.0) || !isfinite(d);
    if (bad) {
      if (threadIdx.x == 0) record_error(err, DDG_ERR_NOT_SPD, sub, blk, row0 + t);
      d = 1.0;
    }
    double nv[4];
    int cnt = 0;
    for (int idx = threadIdx.x; idx < w * w; idx += NT, ++cnt) {
      const int i = idx / w, c = idx % w;
      const double aic = piv[i * ldp + c];
      const double ait = piv[i * ldp + t];
      const double atc = piv[t * ldp + c];
      double v;
      if (i == t && c == t) v = 1.0 / d;
      else if (i == t) v = atc / d;
      else if (c == t) v = -ait / d;
      else v = aic - ait * atc / d;
      nv[cnt] = v;
    }
    __syncthreads();
    cnt = 0;
    for (int idx = threadIdx.x; idx < w * w; idx += NT, ++cnt) piv[(idx / w) * ldp + idx % w] = nv[cnt];
    __syncthreads();
  }
}

// In-place blocked Gauss-Jordan inverse of the SPD b x b row-major matrix A (ld = b)
// by one workgroup.  Rp is an LDS buffer of nb * b doubles, piv nb*(nb+1).
template <int NT, int NB>
__device__ void gj_invert_wg(double* __restrict__ A, int b, double* Rp, double* piv, int32_t* err,
                             int sub, int blk) {
  constexpr int LDP = NB + 1;
  for (int P0 = 0; P0 < b; P0 += NB) {
    const int w = min(NB, b - P0);
    for (int idx = threadIdx.x; idx < w * w; idx += NT)
      piv[(idx / w) * LDP + idx % w] = A[(int64_t)(P0 + idx / w) * b + P0 + idx % w];
    __syncthreads();
    gj_small<NT>(piv, w, LDP, err, sub, blk, P0);
    // new row panel: R = Pinv * A[P, c] for c outside P (written in place and kept in LDS)
    for (int c = threadIdx.x; c < b; c += NT) {
      if (c >= P0 && c < P0 + w) continue;
      double old[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) old[u] = (u < w) ? A[(int64_t)(P0 + u) * b + c] : 0.0;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < w) {
          double s = 0.0;
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (u < w) s += piv[t * LDP + u] * old[u];
          Rp[t * b + c] = s;
          A[(int64_t)(P0 + t) * b + c] = s;
        }
      }
    }
    __syncthreads();
    // trailing update, 4 columns per thread: A[i, c] -= A[i, P] R[P, c]
    const int c4n = (b + 3) / 4;
    for (int idx = threadIdx.x; idx < b * c4n; idx += NT) {
      const int i = idx / c4n;
      if (i >= P0 && i < P0 + w) continue;
      const int c0 = (idx % c4n) * 4;
      double colp[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) colp[u] = (u < w) ? A[(int64_t)i * b + P0 + u] : 0.0;
      for (int cc = 0; cc < 4; ++cc) {
        const int c = c0 + cc;
        if (c >= b || (c >= P0 && c < P0 + w)) continue;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < NB; ++u)
          if (u < w) s += colp[u] * Rp[u * b + c];
        A[(int64_t)i * b + c] -= s;
      }
    }
    __syncthreads();
    // new column panel: A[i, P] = -A[i, P] Pinv, and the pivot block itself
    for (int i = threadIdx.x; i < b; i += NT) {
      if (i >= P0 && i < P0 + w) {
        for (int t = 0; t < w; ++t) A[(int64_t)i * b + P0 + t] = piv[(i - P0) * LDP + t];
        continue;
      }
      double old[NB];
#pragma unroll
      for (int u = 0; u < NB; ++u) old[u] = (u < w) ? A[(int64_t)i * b + P0 + u] : 0.0;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < w) {
          double s = 0.0;
#pragma unroll
          for (int u = 0; u < NB; ++u)
            if (u < w) s += old[u] * piv[u * LDP + t];
          A[(int64_t)i * b + P0 + t] = -s;
        }
      }
    }
    __syncthreads();
  }
}

// Pack the lower triangle of a symmetric b x b row-major matrix (ld) into T x T tiles
// (layout of symv_tile.hpp).
template <class FT, int T, int NT>
__device__ inline void pack_tiles_wg(const double* __restrict__ A, int64_t ld, int b, FT* __restrict__ out) {
  const int nt = (b + T - 1) / T;
  const int64_t total = (int64_t)nt * (nt + 1) / 2 * T * T;
  for (int64_t idx = threadIdx.x; idx < total; idx += NT) {
    const int t = (int)(idx / (T * T));
    int rr, cc;
    tile_rc<FT, T>((int)(idx % (T * T)), rr, cc);
    int I, J;
    tile_ij(t, I, J);
    const int row = I * T + rr;
    const int col = J * T + cc;
    double v = 0.0;
    if (row < b && col < b) v = (row >= col) ? A[(int64_t)row * ld + col] : A[(int64_t)col * ld + row];
    out[idx] = Store<FT>::from(v);
  }
}

// ---------------------------------------------------------------------------
// Local factorisation (twisted block LDL^T, see kernels_sweep.hip): for each
// subdomain a top chain (levels 0..m-1, couplings to the level below) and a
// bottom chain (levels K-1..m+1, couplings to the level above) run as two
// independent workgroups; a second kernel forms and inverts the middle level.

constexpr int kFacThreads = 256;
constexpr int kFacNB = 16;

struct FactorArgs {
  int32_t first_sub;
  const int64_t* set_ptr;
  const int32_t* sub_blk_ptr;
  const int32_t* blk_start;
  const int32_t* blk_size;
  const int64_t* blk_foff;
  const int32_t* lo_col;
  const int64_t* lo_pos;
  int32_t cl;
  const int32_t* up_col;
  const int64_t* up_pos;
  int32_t cu;
  const int64_t* in_ptr;
  const int32_t* in_col;
  const int64_t* in_pos;
  const double* val;
  double* scratch;
  int64_t bmax2;
  void* fac;
  int32_t* err;
};

// Sm = D_k (row-major b x b) from the same-level entries of rows row0..row0+b-1.
__device__ inline void load_diag_block(double* Sm, int b, int bs, int64_t row0, const FactorArgs& a) {
  for (int idx = threadIdx.x; idx < b * b; idx += kFacThreads) Sm[idx] = 0.0;
  __syncthreads();
  for (int jj = threadIdx.x; jj < b; jj += kFacThreads) {
    const int64_t row = row0 + jj;
    for (int64_t t = a.in_ptr[row]; t < a.in_ptr[row + 1]; ++t)
      Sm[(int64_t)jj * b + (a.in_col[t] - bs)] = a.val[a.in_pos[t]];
  }
  __syncthreads();
}

// Sm -= C X C^T, where C (b x bp) holds the couplings of rows row0.. to the level
// starting at bsp (ELL slots ccol/cpos, cc per row) and X is bp x bp.
__device__ inline void schur_update(double* Sm, int b, const double* X, int bp, int bsp, double* Tm,
                                    const int32_t* ccol, const int64_t* cpos, int cc, int64_t row0,
                                    const double* val) {
  for (int idx = threadIdx.x; idx < bp * b; idx += kFacThreads) {
    const int pp = idx / b, c = idx % b;
    const int64_t row = row0 + c;
    double acc = 0.0;
    for (int q = 0; q < cc; ++q) {
      const int col = ccol[row * cc + q];
      if (col >= 0) acc += X[(int64_t)pp * bp + (col - bsp)] * val[cpos[row * cc + q]];
    }
    Tm[idx] = acc;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < b * b; idx += kFacThreads) {
    const int r = idx / b, c = idx % b;
    const int64_t row = row0 + r;
    double acc = 0.0;
    for (int q = 0; q < cc; ++q) {
      const int col = ccol[row * cc + q];
      if (col >= 0) acc += val[cpos[row * cc + q]] * Tm[(int64_t)(col - bsp) * b + c];
    }
    Sm[idx] -= acc;
  }
  __syncthreads();
}

template <class FT, int T, int NB>
__global__ void __launch_bounds__(kFacThreads) k_local_factor_chain(FactorArgs a) {
  extern __shared__ __align__(16) double fsm[];
  double* piv = fsm;                                 // NB*(NB+1)
  double* Rp = fsm + NB * (NB + 1);                  // NB * bmax
  const int slot = blockIdx.x >> 1, chain = blockIdx.x & 1;
  const int sub = a.first_sub + slot;
  double* buf = a.scratch + (int64_t)(2 * slot + chain) * 3 * a.bmax2;
  double* X = buf;
  double* Tm = buf + a.bmax2;
  double* Sm = buf + 2 * a.bmax2;
  const int64_t s0 = a.set_ptr[sub];
  const int kb0 = a.sub_blk_ptr[sub];
  const int K = a.sub_blk_ptr[sub + 1] - kb0;
  const int m = (K - 1) / 2;
  const int steps = chain == 0 ? m : K - 1 - m;
  FT* fac = static_cast<FT*>(a.fac);
  for (int j = 0; j < steps; ++j) {
    const int k = chain == 0 ? j : K - 1 - j;
    const int bs = a.blk_start[kb0 + k];
    const int b = a.blk_size[kb0 + k];
    load_diag_block(Sm, b, bs, s0 + bs, a);
    if (j > 0) {
      const int kp = chain == 0 ? k - 1 : k + 1;
      if (chain == 0)
        schur_update(Sm, b, X, a.blk_size[kb0 + kp], a.blk_start[kb0 + kp], Tm, a.lo_col, a.lo_pos, a.cl,
                     s0 + bs, a.val);
      else
        schur_update(Sm, b, X, a.blk_size[kb0 + kp], a.blk_start[kb0 + kp], Tm, a.up_col, a.up_pos, a.cu,
                     s0 + bs, a.val);
    }
    gj_invert_wg<kFacThreads, NB>(Sm, b, Rp, piv, a.err, sub, k);
    pack_tiles_wg<FT, T, kFacThreads>(Sm, b, b, fac + a.blk_foff[kb0 + k]);
    __syncthreads();
    double* tmp = X;
    X = Sm;
    Sm = tmp;
  }
}

template <class FT, int T, int NB>
__global__ void __launch_bounds__(kFacThreads) k_local_factor_mid(FactorArgs a) {
  extern __shared__ __align__(16) double fsm[];
  double* piv = fsm;
  double* Rp = fsm + NB * (NB + 1);
  const int slot = blockIdx.x;
  const int sub = a.first_sub + slot;
  const int64_t s0 = a.set_ptr[sub];
  const int kb0 = a.sub_blk_ptr[sub];
  const int K = a.sub_blk_ptr[sub + 1] - kb0;
  const int m = (K - 1) / 2;
  const int nB = K - 1 - m;
  double* bufA = a.scratch + (int64_t)(2 * slot) * 3 * a.bmax2;
  double* bufB = a.scratch + (int64_t)(2 * slot + 1) * 3 * a.bmax2;
  // after n chain steps the chain's last inverse sits in slot 0 (n even) or slot 2 (n odd)
  const double* XA = bufA + ((m & 1) ? 2 : 0) * a.bmax2;
  const double* XB = bufB + ((nB & 1) ? 2 : 0) * a.bmax2;
  double* Tm = bufA + a.bmax2;
  double* Sm = bufA + ((m & 1) ? 0 : 2) * a.bmax2;
  const int bs = a.blk_start[kb0 + m];
  const int b = a.blk_size[kb0 + m];
  load_diag_block(Sm, b, bs, s0 + bs, a);
  if (m > 0)
    schur_update(Sm, b, XA, a.blk_size[kb0 + m - 1], a.blk_start[kb0 + m - 1], Tm, a.lo_col, a.lo_pos, a.cl,
                 s0 + bs, a.val);
  if (nB > 0)
    schur_update(Sm, b, XB, a.blk_size[kb0 + m + 1], a.blk_start[kb0 + m + 1], Tm, a.up_col, a.up_pos, a.cu,
                 s0 + bs, a.val);
  gj_invert_wg<kFacThreads, NB>(Sm, b, Rp, piv, a.err, sub, m);
  FT* fac = static_cast<FT*>(a.fac);
  pack_tiles_wg<FT, T, kFacThreads>(Sm, b, b, fac + a.blk_foff[kb0 + m]);
}

__global__ void k_gather_vals(const int64_t* __restrict__ pos, const double* __restrict__ val,
                              double* __restrict__ out, int64_t m) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = pos[i] >= 0 ? val[pos[i]] : 0.0;
}

// ---------------------------------------------------------------------------
// Coarse inverse: blocked Gauss-Jordan over the whole device, one dense block
// per independent system (the last grid dimension selects the system).

constexpr int kCNB = 64;

struct CoarseBlocks {
  double* A;               // dense blocks
  const int64_t* a0_off;   // element offset of each block
  const int32_t* n;        // order of each block
  double* pinv;            // per system kCNB x kCNB
  double* Rbuf;            // per system kCNB x (order), at kCNB * cblk_off
  const int64_t* cblk_off;
};

__global__ void __launch_bounds__(256) k_cgj_pivot(CoarseBlocks cb, int P0, int32_t* err) {
  const int sys = blockIdx.x;
  const int64_t N = cb.n[sys];
  if (P0 >= N) return;
  const int w = (int)min<int64_t>(kCNB, N - P0);
  double* A = cb.A + cb.a0_off[sys];
  double* pinv = cb.pinv + (int64_t)sys * kCNB * kCNB;
  __shared__ double piv[kCNB * (kCNB + 1)];
  for (int idx = threadIdx.x; idx < w * w; idx += 256)
    piv[(idx / w) * (kCNB + 1) + idx % w] = A[(int64_t)(P0 + idx / w) * N + P0 + idx % w];
  __syncthreads();
  for (int t = 0; t < w; ++t) {
    double d = piv[t * (kCNB + 1) + t];
    if (!(d > 0.0) || !isfinite(d)) {
      if (threadIdx.x == 0) record_error(err, DDG_ERR_NOT_SPD, -1, sys, P0 + t);
      d = 1.0;
    }
    double nv[16];
    int cnt = 0;
    for (int idx = threadIdx.x; idx < w * w; idx += 256, ++cnt) {
      const int i = idx / w, c = idx % w;
      const double aic = piv[i * (kCNB + 1) + c];
      const double ait = piv[i * (kCNB + 1) + t];
      const double atc = piv[t * (kCNB + 1) + c];
      double v;
      if (i == t && c == t) v = 1.0 / d;
      else if (i == t) v = atc / d;
      else if (c == t) v = -ait / d;
      else v = aic - ait * atc / d;
      nv[cnt] = v;
    }
    __syncthreads();
    cnt = 0;
    for (int idx = threadIdx.x; idx < w * w; idx += 256, ++cnt)
      piv[(idx / w) * (kCNB + 1) + idx % w] = nv[cnt];
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < w * w; idx += 256) pinv[idx] = piv[(idx / w) * (kCNB + 1) + idx % w];
}

// row panel R = Pinv A[P, :] for columns outside P; written to Rbuf and in place
__global__ void k_cgj_row(CoarseBlocks cb, int P0) {
  const int sys = blockIdx.y;
  const int64_t N = cb.n[sys];
  if (P0 >= N) return;
  const int w = (int)min<int64_t>(kCNB, N - P0);
  double* A = cb.A + cb.a0_off[sys];
  const double* pinv = cb.pinv + (int64_t)sys * kCNB * kCNB;
  double* Rbuf = cb.Rbuf + kCNB * cb.cblk_off[sys];
  __shared__ double pv[kCNB * kCNB];
  for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) pv[idx] = pinv[idx];
  __syncthreads();
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N || (c >= P0 && c < P0 + w)) return;
  double old[kCNB];
#pragma unroll
  for (int u = 0; u < kCNB; ++u) old[u] = (u < w) ? A[(int64_t)(P0 + u) * N + c] : 0.0;
  for (int t = 0; t < w; ++t) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kCNB; ++u)
      if (u < w) s += pv[t * w + u] * old[u];
    Rbuf[(int64_t)t * N + c] = s;
    A[(int64_t)(P0 + t) * N + c] = s;
  }
}

// trailing update on 64 x 64 output tiles: A[i, c] -= A[i, P] R[P, c]
__global__ void __launch_bounds__(256) k_cgj_update(CoarseBlocks cb, int P0) {
  const int sys = blockIdx.z;
  const int64_t N = cb.n[sys];
  const int64_t i0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
  if (P0 >= N || i0 >= N || c0 >= N) return;
  const int w = (int)min<int64_t>(kCNB, N - P0);
  double* A = cb.A + cb.a0_off[sys];
  const double* Rbuf = cb.Rbuf + kCNB * cb.cblk_off[sys];
  constexpr int UC = 32;
  __shared__ double cp[64][UC + 1];   // column panel rows of this tile
  __shared__ double rp[UC][64 + 1];   // row panel columns of this tile
  const int tr = threadIdx.x / 16, tc = threadIdx.x % 16;
  double acc[4][4] = {};
  for (int u0 = 0; u0 < w; u0 += UC) {
    for (int idx = threadIdx.x; idx < 64 * UC; idx += 256) {
      const int r = idx / UC, u = idx % UC;
      const int64_t i = i0 + r;
      cp[r][u] = (u0 + u < w && i < N) ? A[i * N + P0 + u0 + u] : 0.0;
      const int uu = idx / 64, cc = idx % 64;
      const int64_t c = c0 + cc;
      rp[uu][cc] = (u0 + uu < w && c < N) ? Rbuf[(int64_t)(u0 + uu) * N + c] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int u = 0; u < UC; ++u) {
      double av[4], bv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        av[x] = cp[tr * 4 + x][u];
        bv[x] = rp[u][tc * 4 + x];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] += av[x] * bv[y];
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    const int64_t i = i0 + tr * 4 + x;
    if (i >= N || (i >= P0 && i < P0 + w)) continue;
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int64_t c = c0 + tc * 4 + y;
      if (c >= N || (c >= P0 && c < P0 + w)) continue;
      A[i * N + c] -= acc[x][y];
    }
  }
}

// column panel A[i, P] = -A[i, P] Pinv (rows outside P) and the pivot block itself
__global__ void k_cgj_col(CoarseBlocks cb, int P0) {
  const int sys = blockIdx.y;
  const int64_t N = cb.n[sys];
  if (P0 >= N) return;
  const int w = (int)min<int64_t>(kCNB, N - P0);
  double* A = cb.A + cb.a0_off[sys];
  const double* pinv = cb.pinv + (int64_t)sys * kCNB * kCNB;
  __shared__ double pv[kCNB * kCNB];
  for (int idx = threadIdx.x; idx < w * w; idx += blockDim.x) pv[idx] = pinv[idx];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  if (i >= P0 && i < P0 + w) {
    for (int t = 0; t < w; ++t) A[i * N + P0 + t] = pv[(i - P0) * w + t];
    return;
  }
  double old[kCNB];
#pragma unroll
  for (int u = 0; u < kCNB; ++u) old[u] = (u < w) ? A[i * N + P0 + u] : 0.0;
  for (int t = 0; t < w; ++t) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < kCNB; ++u)
      if (u < w) s += old[u] * pv[u * w + t];
    A[i * N + P0 + t] = -s;
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

template <class FT, int T>
void launch_factor_t(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  const int64_t bmax2 = (int64_t)S.max_blk * S.max_blk;
  // bound the scratch: at most `batch` subdomains in flight per launch
  const int64_t per = 2 * 3 * bmax2 * 8;
  int batch = (int)std::min<int64_t>(S.n_parts, std::max<int64_t>(1, ((int64_t)6 << 30) / per));
  if ((int64_t)h.fac_scratch.bytes < per * batch) h.fac_scratch.alloc(per * batch);
  FactorArgs a;
  a.set_ptr = h.set_ptr.as<int64_t>();
  a.sub_blk_ptr = h.sub_blk_ptr.as<int32_t>();
  a.blk_start = h.blk_start.as<int32_t>();
  a.blk_size = h.blk_size.as<int32_t>();
  a.blk_foff = h.blk_foff.as<int64_t>();
  a.lo_col = h.lo_col.as<int32_t>();
  a.lo_pos = h.lo_pos.as<int64_t>();
  a.cl = S.cl;
  a.up_col = h.up_col.as<int32_t>();
  a.up_pos = h.up_pos.as<int64_t>();
  a.cu = S.cu;
  a.in_ptr = h.in_ptr.as<int64_t>();
  a.in_col = h.in_col.as<int32_t>();
  a.in_pos = h.in_pos.as<int64_t>();
  a.val = h.val.as<double>();
  a.scratch = h.fac_scratch.as<double>();
  a.bmax2 = bmax2;
  a.fac = h.fac.p;
  a.err = h.err_flag.as<int32_t>();
  // panel width 16 when its row panel fits on chip, else 8 (wide levels)
  auto lds_for = [&](int nb) { return sizeof(double) * ((size_t)nb * (nb + 1) + (size_t)nb * S.max_blk); };
  const bool wide = (int64_t)lds_for(kFacNB) > h.dev_lds_limit - 1024;
  const size_t lds = wide ? lds_for(8) : lds_for(kFacNB);
  DDG_REQUIRE((int64_t)lds <= h.dev_lds_limit - 1024, DDG_ERR_UNSUPPORTED, "local level too wide for the factorisation");
  auto kc = wide ? k_local_factor_chain<FT, T, 8> : k_local_factor_chain<FT, T, kFacNB>;
  auto km = wide ? k_local_factor_mid<FT, T, 8> : k_local_factor_mid<FT, T, kFacNB>;
  if (lds > 65536) {
    DDG_HIP(hipFuncSetAttribute((const void*)kc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    DDG_HIP(hipFuncSetAttribute((const void*)km, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  for (int first = 0; first < S.n_parts; first += batch) {
    a.first_sub = first;
    const int cnt = std::min(batch, S.n_parts - first);
    hipLaunchKernelGGL(kc, dim3(2 * cnt), dim3(kFacThreads), lds, s, a);
    hipLaunchKernelGGL(km, dim3(cnt), dim3(kFacThreads), lds, s, a);
    DDG_HIP(hipGetLastError());
  }
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
  DDG_REQUIRE(h.k <= kMaxKq, DDG_ERR_UNSUPPORTED, "at most 32 generating vectors");
  DevBuf work;
  work.alloc((size_t)S.n * h.k * sizeof(double));
  hipLaunchKernelGGL(k_coarse_qr, dim3(S.n_parts), dim3(kQrThreads), 0, s, h.own_ptr.as<int64_t>(),
                     h.own_idx.as<int32_t>(), h.F.as<double>(), S.n, h.k, h.opt.rank_tol,
                     work.as<double>(), h.Q.as<double>(), h.kcnt_d.as<int32_t>(), h.err_flag.as<int32_t>());
  DDG_HIP(hipGetLastError());
  DDG_HIP(hipStreamSynchronize(s));
}

void launch_galerkin(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  DDG_HIP(hipMemsetAsync(h.A0.p, 0, (size_t)h.a0_off[h.nb] * sizeof(double), s));
  hipLaunchKernelGGL(k_galerkin, dim3(S.n_parts), dim3(kGalThreads), 0, s, h.own_ptr.as<int64_t>(),
                     h.own_idx.as<int32_t>(), h.nbr_ptr.as<int32_t>(), h.nbr_idx.as<int32_t>(),
                     h.part.as<int32_t>(), h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(),
                     h.Q.as<double>(), h.k, h.rowptr.as<int64_t>(), h.col.as<int32_t>(),
                     h.val.as<double>(), h.sub_inst.as<int32_t>(), h.cblk_off_d.as<int64_t>(),
                     h.cblk_n_d.as<int32_t>(), h.a0_off_d.as<int64_t>(), h.A0.as<double>());
  DDG_HIP(hipGetLastError());
}

void launch_coarse_invert(Handle& h, hipStream_t s) {
  const int64_t total = h.a0_off[h.nb];
  int64_t nmax = 0;
  for (int32_t b = 0; b < h.nb; ++b) nmax = std::max<int64_t>(nmax, h.cblk_n[b]);
  DevBuf work;
  work.alloc(((size_t)kCNB * kCNB * h.nb + (size_t)kCNB * h.nc_pad) * sizeof(double));
  // the inverse is formed in a copy so that A0 stays available for export
  DevBuf inv;
  inv.alloc((size_t)total * sizeof(double));
  DDG_HIP(hipMemcpyAsync(inv.p, h.A0.p, (size_t)total * sizeof(double), hipMemcpyDeviceToDevice, s));
  CoarseBlocks cb;
  cb.A = inv.as<double>();
  cb.a0_off = h.a0_off_d.as<int64_t>();
  cb.n = h.cblk_n_d.as<int32_t>();
  cb.pinv = work.as<double>();
  cb.Rbuf = cb.pinv + (int64_t)kCNB * kCNB * h.nb;
  cb.cblk_off = h.cblk_off_d.as<int64_t>();
  const unsigned tiles = (unsigned)((nmax + 63) / 64);
  const unsigned nb = (unsigned)h.nb;
  for (int P0 = 0; P0 < nmax; P0 += kCNB) {
    hipLaunchKernelGGL(k_cgj_pivot, dim3(nb), dim3(256), 0, s, cb, P0, h.err_flag.as<int32_t>());
    hipLaunchKernelGGL(k_cgj_row, dim3((unsigned)((nmax + 127) / 128), nb), dim3(128), 0, s, cb, P0);
    hipLaunchKernelGGL(k_cgj_update, dim3(tiles, tiles, nb), dim3(256), 0, s, cb, P0);
    hipLaunchKernelGGL(k_cgj_col, dim3((unsigned)((nmax + 127) / 128), nb), dim3(128), 0, s, cb, P0);
  }
  const int64_t elems = h.ntiles * 64 * 64;
  hipLaunchKernelGGL(k_pack_coarse, dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s, cb.A,
                     h.a0_off_d.as<int64_t>(), h.cblk_n_d.as<int32_t>(), h.tile_inst.as<int32_t>(),
                     h.tile_base_d.as<int64_t>(), h.ntiles, h.A0inv_t.as<double>());
  DDG_HIP(hipGetLastError());
  DDG_HIP(hipStreamSynchronize(s));
}

void launch_local_factor(Handle& h, hipStream_t s) {
  switch (h.opt.precision) {
    case DDG_MIXED_FP32: launch_factor_p<float>(h, s); break;
    case DDG_MIXED_BF16: launch_factor_p<__hip_bfloat16>(h, s); break;
    default: launch_factor_p<double>(h, s); break;
  }
}

void launch_refresh_couplings(Handle& h, hipStream_t s) {
  const int64_t nlo = (int64_t)h.S.lo_pos.size(), nup = (int64_t)h.S.up_pos.size();
  if (nlo)
    hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((nlo + 255) / 256)), dim3(256), 0, s,
                       h.lo_pos.as<int64_t>(), h.val.as<double>(), h.lo_val.as<double>(), nlo);
  if (nup)
    hipLaunchKernelGGL(k_gather_vals, dim3((unsigned)((nup + 255) / 256)), dim3(256), 0, s,
                       h.up_pos.as<int64_t>(), h.val.as<double>(), h.up_val.as<double>(), nup);
  DDG_HIP(hipGetLastError());
}

}  // namespace ddg
