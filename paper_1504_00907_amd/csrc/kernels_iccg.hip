// Inexact coarse solve (Section 7, the timed 3D runs): CG on A0 y = b0 from
// y = 0, preconditioned by the zero-fill incomplete Cholesky factor of A0, and
// stopped at ||r|| <= ic_tol ||b0|| or after ic_maxit iterations.
//
// Pattern.  A0 = R0 A R0^T (Section 4) couples the coarse unknowns of two
// subdomains only when A couples the subdomains, so its pattern is the block
// pattern of coupled subdomains.  The factor keeps that pattern structurally: every
// entry of a block (I, J), J <= I coupled, is computed, zero values included.
//
// Factorisation (k_ic_factor, one workgroup per system).  Block rows I in
// ascending order; in row I the coupled blocks J < I in ascending order, then the
// diagonal block.  Each entry follows the zero-fill rule
//     L_ij = (A_ij - sum_{c < j, (i,c) and (j,c) in the pattern} L_ic L_jc) / L_jj,
//     L_ii = sqrt(A_ii - sum_{c < i} L_ic^2),
// with the sum taken block by block (coupled K in ascending order, then the
// columns of the block); a K contributes when it is coupled to both I and J.  The
// inverse of every diagonal block is stored (32 x 32 slot per subdomain) so that
// the triangular solves apply it as a small product.
//
// Solve (k_ic_pcg, one workgroup of 1024 threads per system, the whole inner CG).
// The products with A0 read the dense blocks of the coupled subdomains.  The
// forward solve L w = r goes level by level over the lower block graph (a block's
// level exceeds those of the coupled blocks before it), the backward solve
// L^T z = w level by level in reverse; within a level each row is one thread.
#include "common.hpp"
#include "device_util.hpp"

namespace ddg {

namespace {

constexpr int kIcFacThreads = 256;
constexpr int kIcThreads = 1024;
constexpr int kIcSlot = 32 * 32;   // inverse of one diagonal block

struct IcArgs {
  const int32_t* sub_off;   // nb + 1: subdomains of each system
  const int32_t* nbr_ptr;   // coupled subdomains of each subdomain (ascending, itself included)
  const int32_t* nbr_idx;
  const int32_t* kcnt;
  const int64_t* koff;      // first coarse row of each subdomain (padded numbering)
  const int64_t* cblk_off;  // first coarse row of each system
  const int32_t* cblk_n;
  const int64_t* a0_off;    // dense N x N block of each system, row-major
  const double* A0;
  double* L;                // the factor's blocks, in A0's layout
  double* D;                // per subdomain: inverse of its diagonal block of L (row-major, 32 x 32)
  int32_t* mark;            // per subdomain: factorisation scratch
  int32_t* err;
};

struct IcSolveArgs {
  IcArgs f;
  const int32_t* sys_lvl;   // nb + 1: levels of each system in lvl_ptr
  const int32_t* lvl_ptr;   // rows of each level in lvl_rows
  const int32_t* lvl_rows;  // coarse rows (padded numbering), level by level
  const int32_t* row_sub;   // subdomain of every coarse row (-1 on padding)
  const CgState* st;        // skip systems that have stopped (null: none)
  const double* b0;         // right-hand side (padded numbering)
  double* y;                // solution
  double* w;                // work: r, z, p, q, t (nc_pad each)
  int64_t nc_pad;
  double tol;
  int32_t maxit;
  int32_t* iters;           // per system: inner iterations added
};

__device__ inline void ic_record(int32_t* err, int row) {
  if (atomicCAS(err, 0, DDG_ERR_NOT_SPD) == 0) {
    err[1] = -1;
    err[2] = -1;
    err[3] = row;
  }
}

__global__ void __launch_bounds__(kIcFacThreads) k_ic_factor(IcArgs a) {
  const int b = blockIdx.x;
  const int N = a.cblk_n[b];
  if (N == 0) return;
  const double* A = a.A0 + a.a0_off[b];
  double* L = a.L + a.a0_off[b];
  const int64_t c0 = a.cblk_off[b];
  __shared__ double U[32 * 32];
  __shared__ double piv;
  const int tid = threadIdx.x;
  for (int I = a.sub_off[b]; I < a.sub_off[b + 1]; ++I) {
    const int kI = a.kcnt[I];
    const int oI = (int)(a.koff[I] - c0);
    const int n0 = a.nbr_ptr[I], n1 = a.nbr_ptr[I + 1];
    for (int t = n0 + tid; t < n1; t += kIcFacThreads) a.mark[a.nbr_idx[t]] = I + 1;
    __syncthreads();
    // blocks (I, J), J < I coupled, in ascending J
    for (int t = n0; t < n1; ++t) {
      const int J = a.nbr_idx[t];
      if (J >= I) break;
      const int kJ = a.kcnt[J];
      const int oJ = (int)(a.koff[J] - c0);
      for (int e = tid; e < kI * kJ; e += kIcFacThreads) {
        const int i = e / kJ, j = e % kJ;
        double s = A[(int64_t)(oI + i) * N + oJ + j];
        for (int u = a.nbr_ptr[J]; u < a.nbr_ptr[J + 1]; ++u) {
          const int K = a.nbr_idx[u];
          if (K >= J) break;
          if (a.mark[K] != I + 1) continue;
          const int oK = (int)(a.koff[K] - c0), kK = a.kcnt[K];
          const double* li = L + (int64_t)(oI + i) * N + oK;
          const double* lj = L + (int64_t)(oJ + j) * N + oK;
          for (int c = 0; c < kK; ++c) s -= li[c] * lj[c];
        }
        U[i * 32 + j] = s;
      }
      __syncthreads();
      for (int j = 0; j < kJ; ++j) {
        const double* lj = L + (int64_t)(oJ + j) * N + oJ;
        for (int i = tid; i < kI; i += kIcFacThreads) {
          const double* li = L + (int64_t)(oI + i) * N + oJ;
          double s = U[i * 32 + j];
          for (int c = 0; c < j; ++c) s -= li[c] * lj[c];
          L[(int64_t)(oI + i) * N + oJ + j] = s / lj[j];
        }
        __syncthreads();
      }
    }
    // the diagonal block: updates from the coupled blocks before it, then its own Cholesky
    for (int e = tid; e < kI * kI; e += kIcFacThreads) {
      const int i = e / kI, j = e % kI;
      if (j > i) continue;
      double s = A[(int64_t)(oI + i) * N + oI + j];
      for (int t = n0; t < n1; ++t) {
        const int K = a.nbr_idx[t];
        if (K >= I) break;
        const int oK = (int)(a.koff[K] - c0), kK = a.kcnt[K];
        const double* li = L + (int64_t)(oI + i) * N + oK;
        const double* lj = L + (int64_t)(oI + j) * N + oK;
        for (int c = 0; c < kK; ++c) s -= li[c] * lj[c];
      }
      U[i * 32 + j] = s;
    }
    __syncthreads();
    for (int j = 0; j < kI; ++j) {
      const double* lj = L + (int64_t)(oI + j) * N + oI;
      if (tid == 0) {
        double d = U[j * 32 + j];
        for (int c = 0; c < j; ++c) d -= lj[c] * lj[c];
        if (!(d > 0.0) || !isfinite(d)) {
          ic_record(a.err, (int)(c0 + oI + j));
          d = 1.0;
        }
        piv = sqrt(d);
        L[(int64_t)(oI + j) * N + oI + j] = piv;
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < kI; i += kIcFacThreads) {
        const double* li = L + (int64_t)(oI + i) * N + oI;
        double s = U[i * 32 + j];
        for (int c = 0; c < j; ++c) s -= li[c] * lj[c];
        L[(int64_t)(oI + i) * N + oI + j] = s / piv;
      }
      __syncthreads();
    }
    // inverse of the diagonal block by forward substitution, one column per thread
    double* Dm = a.D + (int64_t)I * kIcSlot;
    for (int c = tid; c < kI; c += kIcFacThreads) {
      for (int r = 0; r < kI; ++r) {
        if (r < c) {
          Dm[r * 32 + c] = 0.0;
          continue;
        }
        const double* lr = L + (int64_t)(oI + r) * N + oI;
        double s = r == c ? 1.0 : 0.0;
        for (int t = c; t < r; ++t) s -= lr[t] * Dm[t * 32 + c];
        Dm[r * 32 + c] = s / lr[r];
      }
    }
    __syncthreads();
  }
}

// sum of v over the workgroup, the same value in every thread (fixed order)
__device__ inline double ic_sum(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kIcThreads / 64; ++i) s += red[i];
  __syncthreads();
  return s;
}

// z = (L L^T)^{-1} r on the rows of system b (t: scratch); local row numbering
__device__ void ic_apply(const IcSolveArgs& a, int b, int N, int64_t c0, const double* L, const double* r,
                         double* z, double* t) {
  const IcArgs& f = a.f;
  const int l0 = a.sys_lvl[b], l1 = a.sys_lvl[b + 1];
  // forward: w = L^{-1} r, level by level (w is kept in z)
  for (int l = l0; l < l1; ++l) {
    for (int q = a.lvl_ptr[l] + threadIdx.x; q < a.lvl_ptr[l + 1]; q += kIcThreads) {
      const int i = (int)(a.lvl_rows[q] - c0);
      const int I = a.row_sub[c0 + i];
      double s = r[i];
      for (int u = f.nbr_ptr[I]; u < f.nbr_ptr[I + 1]; ++u) {
        const int J = f.nbr_idx[u];
        if (J >= I) break;
        const int oJ = (int)(f.koff[J] - c0), kJ = f.kcnt[J];
        const double* li = L + (int64_t)i * N + oJ;
        for (int c = 0; c < kJ; ++c) s -= li[c] * z[oJ + c];
      }
      t[i] = s;
    }
    __syncthreads();
    for (int q = a.lvl_ptr[l] + threadIdx.x; q < a.lvl_ptr[l + 1]; q += kIcThreads) {
      const int i = (int)(a.lvl_rows[q] - c0);
      const int I = a.row_sub[c0 + i];
      const int oI = (int)(f.koff[I] - c0), ii = i - oI;
      const double* d = f.D + (int64_t)I * kIcSlot + ii * 32;
      double s = 0.0;
      for (int c = 0; c <= ii; ++c) s += d[c] * t[oI + c];
      z[i] = s;
    }
    __syncthreads();
  }
  // backward: z = L^{-T} w, levels in reverse
  for (int l = l1 - 1; l >= l0; --l) {
    for (int q = a.lvl_ptr[l] + threadIdx.x; q < a.lvl_ptr[l + 1]; q += kIcThreads) {
      const int i = (int)(a.lvl_rows[q] - c0);
      const int I = a.row_sub[c0 + i];
      double s = z[i];
      for (int u = f.nbr_ptr[I + 1] - 1; u >= f.nbr_ptr[I]; --u) {
        const int J = f.nbr_idx[u];
        if (J <= I) break;
        const int oJ = (int)(f.koff[J] - c0), kJ = f.kcnt[J];
        for (int j = 0; j < kJ; ++j) s -= L[(int64_t)(oJ + j) * N + i] * z[oJ + j];
      }
      t[i] = s;
    }
    __syncthreads();
    for (int q = a.lvl_ptr[l] + threadIdx.x; q < a.lvl_ptr[l + 1]; q += kIcThreads) {
      const int i = (int)(a.lvl_rows[q] - c0);
      const int I = a.row_sub[c0 + i];
      const int oI = (int)(f.koff[I] - c0), ii = i - oI, kI = f.kcnt[I];
      const double* d = f.D + (int64_t)I * kIcSlot;
      double s = 0.0;
      for (int c = ii; c < kI; ++c) s += d[c * 32 + ii] * t[oI + c];
      z[i] = s;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kIcThreads) k_ic_pcg(IcSolveArgs a) {
  const int b = blockIdx.x;
  if (a.st && a.st[b].done) return;
  const IcArgs& f = a.f;
  const int N = f.cblk_n[b];
  if (N == 0) return;
  const int64_t c0 = f.cblk_off[b];
  const double* A = f.A0 + f.a0_off[b];
  const double* L = f.L + f.a0_off[b];
  const double* bb = a.b0 + c0;
  double* y = a.y + c0;
  double* r = a.w + c0;
  double* z = r + a.nc_pad;
  double* p = z + a.nc_pad;
  double* q = p + a.nc_pad;
  double* t = q + a.nc_pad;
  __shared__ double red[kIcThreads / 64];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int i = tid; i < N; i += kIcThreads) {
    const double v = bb[i];
    y[i] = 0.0;
    r[i] = v;
    acc += v * v;
  }
  const double b2 = ic_sum(acc, red);
  if (b2 == 0.0) return;
  const double stop = a.tol * sqrt(b2);
  ic_apply(a, b, N, c0, L, r, z, t);
  acc = 0.0;
  for (int i = tid; i < N; i += kIcThreads) {
    p[i] = z[i];
    acc += r[i] * z[i];
  }
  double rho = ic_sum(acc, red);
  int it = 0;
  while (it < a.maxit) {
    // q = A0 p over the coupled blocks of each row's subdomain
    acc = 0.0;
    for (int i = tid; i < N; i += kIcThreads) {
      const int I = a.row_sub[c0 + i];
      const double* ai = A + (int64_t)i * N;
      double s = 0.0;
      for (int u = f.nbr_ptr[I]; u < f.nbr_ptr[I + 1]; ++u) {
        const int J = f.nbr_idx[u];
        const int oJ = (int)(f.koff[J] - c0), kJ = f.kcnt[J];
        for (int c = 0; c < kJ; ++c) s += ai[oJ + c] * p[oJ + c];
      }
      q[i] = s;
      acc += p[i] * s;
    }
    const double pq = ic_sum(acc, red);
    if (!(pq > 0.0) || !isfinite(pq)) break;
    const double alpha = rho / pq;
    acc = 0.0;
    for (int i = tid; i < N; i += kIcThreads) {
      y[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      acc += ri * ri;
    }
    const double rr = ic_sum(acc, red);
    ++it;
    if (sqrt(rr) <= stop) break;
    ic_apply(a, b, N, c0, L, r, z, t);
    acc = 0.0;
    for (int i = tid; i < N; i += kIcThreads) acc += r[i] * z[i];
    const double rho_new = ic_sum(acc, red);
    const double beta = rho_new / rho;
    rho = rho_new;
    for (int i = tid; i < N; i += kIcThreads) p[i] = z[i] + beta * p[i];
    __syncthreads();
  }
  if (tid == 0) a.iters[b] += it;
}

IcArgs ic_args(Handle& h) {
  IcArgs a;
  a.sub_off = h.ic_suboff.as<int32_t>();
  a.nbr_ptr = h.nbr_ptr.as<int32_t>();
  a.nbr_idx = h.nbr_idx.as<int32_t>();
  a.kcnt = h.kcnt_d.as<int32_t>();
  a.koff = h.koff_d.as<int64_t>();
  a.cblk_off = h.cblk_off_d.as<int64_t>();
  a.cblk_n = h.cblk_n_d.as<int32_t>();
  a.a0_off = h.a0_off_d.as<int64_t>();
  a.A0 = h.A0.as<double>();
  a.L = h.icL.as<double>();
  a.D = h.icD.as<double>();
  a.mark = h.ic_mark.as<int32_t>();
  a.err = h.err_flag.as<int32_t>();
  return a;
}

}  // namespace

// Host tables of the inexact coarse solve: per system, its coarse rows grouped by the
// level of their subdomain in the lower block graph (level(I) = 1 + the largest level
// of a coupled J < I), the subdomain of every coarse row, and the factor's buffers.
void prepare_ic(Handle& h, hipStream_t s) {
  const Symbolic& S = h.S;
  const int32_t nb = h.nb;
  std::vector<int32_t> level(S.n_parts, 0), sys_lvl(nb + 1, 0), lvl_ptr(1, 0), lvl_rows;
  std::vector<int32_t> row_sub((size_t)h.nc_pad, -1);
  for (int32_t b = 0; b < nb; ++b) {
    int32_t top = -1;
    for (int32_t I = h.sub_off[b]; I < h.sub_off[b + 1]; ++I) {
      DDG_REQUIRE(h.kcnt[I] <= 32, DDG_ERR_UNSUPPORTED, "incomplete Cholesky coarse solve: at most 32 generating vectors");
      int32_t lv = 0;
      for (int32_t t = S.nbr_ptr[I]; t < S.nbr_ptr[I + 1]; ++t) {
        const int32_t J = S.nbr_idx[t];
        if (J < I) lv = std::max(lv, level[J] + 1);
      }
      level[I] = lv;
      top = std::max(top, lv);
      for (int32_t c = 0; c < h.kcnt[I]; ++c) row_sub[(size_t)(h.koff[I] + c)] = I;
    }
    for (int32_t lv = 0; lv <= top; ++lv) {
      for (int32_t I = h.sub_off[b]; I < h.sub_off[b + 1]; ++I)
        if (level[I] == lv)
          for (int32_t c = 0; c < h.kcnt[I]; ++c) lvl_rows.push_back((int32_t)(h.koff[I] + c));
      lvl_ptr.push_back((int32_t)lvl_rows.size());
    }
    sys_lvl[b + 1] = (int32_t)lvl_ptr.size() - 1;
  }
  if (lvl_rows.empty()) lvl_rows.push_back(0);
  h.ic_sys_lvl.upload(sys_lvl, s);
  h.ic_lvl_ptr.upload(lvl_ptr, s);
  h.ic_lvl_rows.upload(lvl_rows, s);
  h.ic_row_sub.upload(row_sub, s);
  h.ic_suboff.upload(h.sub_off, s);
  h.icL.alloc((size_t)std::max<int64_t>(1, h.a0_off[nb]) * sizeof(double));
  h.icD.alloc((size_t)S.n_parts * kIcSlot * sizeof(double));
  h.icw.alloc((size_t)5 * h.nc_pad * sizeof(double));
  h.ic_mark.alloc((size_t)S.n_parts * sizeof(int32_t));
  h.ic_it.alloc((size_t)nb * sizeof(int32_t));
  DDG_HIP(hipMemsetAsync(h.ic_it.p, 0, (size_t)nb * sizeof(int32_t), s));
}

void launch_ic_factor(Handle& h, hipStream_t s) {
  DDG_HIP(hipMemsetAsync(h.ic_mark.p, 0, (size_t)h.S.n_parts * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_ic_factor, dim3((unsigned)h.nb), dim3(kIcFacThreads), 0, s, ic_args(h));
  DDG_HIP(hipGetLastError());
}

void launch_ic_solve(Handle& h, const CgState* st, const double* b0, double* y, hipStream_t s) {
  IcSolveArgs a;
  a.f = ic_args(h);
  a.sys_lvl = h.ic_sys_lvl.as<int32_t>();
  a.lvl_ptr = h.ic_lvl_ptr.as<int32_t>();
  a.lvl_rows = h.ic_lvl_rows.as<int32_t>();
  a.row_sub = h.ic_row_sub.as<int32_t>();
  a.st = st;
  a.b0 = b0;
  a.y = y;
  a.w = h.icw.as<double>();
  a.nc_pad = h.nc_pad;
  a.tol = h.opt.ic_tol;
  a.maxit = h.opt.ic_maxit;
  a.iters = h.ic_it.as<int32_t>();
  hipLaunchKernelGGL(k_ic_pcg, dim3((unsigned)h.nb), dim3(kIcThreads), 0, s, a);
  DDG_HIP(hipGetLastError());
}

}  // namespace ddg
