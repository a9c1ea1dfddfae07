// Device bodies of the CG steps (Sections 1 and 7: CG from x0 = 0, stop at
// ||r|| <= rtol ||f||), written once and used both by the one-launch-per-step
// kernels (kernels_cg.hip, index = blockIdx) and by the persistent batched solve
// (one workgroup per task).  A chunk body covers the rows [lo[g], hi[g]) of one
// system with the first kCgThreads threads of the workgroup (the others only
// join the barriers) and writes one partial in a fixed order; a scalar body
// sums one system's partials in a fixed order.  So every partial, scalar and
// iterate is the same bit for bit whichever driver runs it.
#pragma once

#include "common.hpp"
#include "device_util.hpp"

namespace ddg {

constexpr int kCgThreads = 256;

struct SegMap {
  const int32_t* seg;   // system of each workgroup (chunk)
  const int64_t* lo;    // first row
  const int64_t* hi;    // end row
  const int32_t* ptr;   // nb+1: partials of system b are [ptr[b], ptr[b+1])
};

// Per-system history of the CG coefficients and residuals (for the Lanczos
// estimates and the fractional iteration count of Section 7): system b owns
// hist[b * 3 * (max_iter + 1) ...], as alpha[j] (j = 0..iters-1), then
// beta[j] (j = 0..iters-2), then ||r_j||^2 (j = 0..iters).
struct Hist {
  double* base;
  int64_t stride;  // max_iter + 1
  __device__ double* alpha(int b) const { return base + (int64_t)b * 3 * stride; }
  __device__ double* beta(int b) const { return base + ((int64_t)b * 3 + 1) * stride; }
  __device__ double* rr(int b) const { return base + ((int64_t)b * 3 + 2) * stride; }
};

__device__ inline uint64_t device_clock() { return wall_clock64(); }

// Sum of v over the first kCgThreads threads (every thread of the workgroup calls
// it; the others pass 0); the same order as block_sum<kCgThreads>; thread 0 holds it.
__device__ inline double cg_block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0 && w < kCgThreads / 64) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kCgThreads / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

__device__ inline double cg_sum_partials(const double* __restrict__ part, int np, double* red) {
  double acc = 0.0;
  if (threadIdx.x < kCgThreads)
    for (int i = threadIdx.x; i < np; i += kCgThreads) acc += part[i];
  return cg_block_sum(acc, red);
}

// first row of this thread in chunk g (past the end for the threads beyond kCgThreads)
__device__ inline int64_t cg_first(const SegMap& m, int g) {
  return threadIdx.x < kCgThreads ? m.lo[g] + threadIdx.x : m.hi[g];
}

__device__ inline void cg_stop(CgState* st, int32_t status) {
  st->status = status;
  st->done = 1;
  st->t_done = device_clock();
}

// x = 0, r = f, partial f.f
__device__ inline void d_cg_init(const SegMap& m, int g, const double* __restrict__ f, double* __restrict__ x,
                                 double* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[kCgThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) {
    double fi = f[i];
    x[i] = 0.0;
    r[i] = fi;
    acc += fi * fi;
  }
  double s = cg_block_sum(acc, red);
  if (threadIdx.x == 0) part[g] = s;
}

__device__ inline void d_cg_init_scalar(CgState* stb, const SegMap& m, int b, const double* __restrict__ part,
                                        double rtol, int max_iter, const Hist& hist) {
  __shared__ double red[kCgThreads / 64];
  CgState* st = stb + b;
  double s = cg_sum_partials(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    hist.rr(b)[0] = s;
    st->iters = 0;
    st->max_iter = max_iter;
    st->status = DDG_OK;
    st->done = 0;
    st->fnorm = sqrt(s);
    st->rr = s;
    st->tol2 = rtol * rtol * s;
    st->rho = st->alpha = st->beta = st->pq = 0.0;
    st->true_rr = 0.0;
    st->t_start = device_clock();
    st->t_done = 0;
    if (!isfinite(s)) {
      st->status = DDG_ERR_INVALID_ARG;
      st->done = 1;
    } else if (s == 0.0) {
      st->done = 1;
    }
    if (st->done) st->t_done = st->t_start;
  }
}

// p = z, partial r.z
__device__ inline void d_copy_dot(const SegMap& m, int g, const double* __restrict__ r, const double* __restrict__ z,
                                  double* __restrict__ p, double* __restrict__ part) {
  __shared__ double red[kCgThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) {
    double zi = z[i];
    p[i] = zi;
    acc += r[i] * zi;
  }
  double s = cg_block_sum(acc, red);
  if (threadIdx.x == 0) part[g] = s;
}

// rho' = r^T z from the partials; beta = rho' / rho (Fletcher-Reeves), or with
// the z^T q partials (part2 non-null) the Polak-Ribiere value
// z^T (r - r_prev) / rho = -alpha z^T q / rho, since r - r_prev = -alpha q.
__device__ inline void d_rho_scalar(CgState* stb, const SegMap& m, int b, const double* __restrict__ part,
                                    const double* __restrict__ part2, int first, const Hist& hist) {
  __shared__ double red[kCgThreads / 64];
  CgState* st = stb + b;
  double s = cg_sum_partials(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  double zq = 0.0;
  if (part2) zq = cg_sum_partials(part2 + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    if (!(s > 0.0) || !isfinite(s)) {
      cg_stop(st, DDG_ERR_BREAKDOWN);
      return;
    }
    if (first) {
      st->rho = s;
    } else {
      const double beta = part2 ? -st->alpha * zq / st->rho : s / st->rho;
      if (!isfinite(beta)) {
        cg_stop(st, DDG_ERR_BREAKDOWN);
        return;
      }
      st->beta = beta;
      st->rho = s;
      hist.beta(b)[st->iters - 1] = beta;
    }
  }
}

// q = A p, partial p.q (L lanes per CSR row, or the diagonals when D.diag is set)
template <int L>
__device__ inline void d_spmv_dot(const SegMap& m, int g, const int64_t* __restrict__ rp,
                                  const int32_t* __restrict__ ci, const double* __restrict__ v, const DiaView& D,
                                  const double* __restrict__ p, double* __restrict__ q, double* __restrict__ part) {
  __shared__ double red[kCgThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[g];
  const int j = threadIdx.x & (L - 1);
  if (L == 1 && D.diag) {
    const DiaSys& sy = D.sys[m.seg[g]];
    for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) {
      const double qi = dia_row_dot(D, sy, p, i);
      q[i] = qi;
      acc += p[i] * qi;
    }
  } else {
    const int64_t i0 = threadIdx.x < kCgThreads ? m.lo[g] + threadIdx.x / L : hi;
    for (int64_t i = i0; i < hi; i += kCgThreads / L) {
      const double qi = row_dot_l<L>(rp, ci, v, p, i, j);
      if (j == 0) {
        q[i] = qi;
        acc += p[i] * qi;
      }
    }
  }
  double s = cg_block_sum(acc, red);
  if (threadIdx.x == 0) part[g] = s;
}

__device__ inline void d_alpha_scalar(CgState* stb, const SegMap& m, int b, const double* __restrict__ part,
                                      const Hist& hist) {
  __shared__ double red[kCgThreads / 64];
  CgState* st = stb + b;
  double s = cg_sum_partials(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    st->pq = s;
    if (!(s > 0.0) || !isfinite(s)) {
      cg_stop(st, DDG_ERR_BREAKDOWN);
      return;
    }
    st->alpha = st->rho / s;
    hist.alpha(b)[st->iters] = st->alpha;
  }
}

// x += alpha p, r -= alpha q, partial r.r
__device__ inline void d_axpy2_dot(const CgState* st, const SegMap& m, int g, double* __restrict__ x,
                                   double* __restrict__ r, const double* __restrict__ p,
                                   const double* __restrict__ q, double* __restrict__ part) {
  __shared__ double red[kCgThreads / 64];
  const double a = st->alpha;
  double acc = 0.0;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) {
    x[i] += a * p[i];
    double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double s = cg_block_sum(acc, red);
  if (threadIdx.x == 0) part[g] = s;
}

__device__ inline void d_conv_scalar(CgState* stb, const SegMap& m, int b, const double* __restrict__ part,
                                     const Hist& hist) {
  __shared__ double red[kCgThreads / 64];
  CgState* st = stb + b;
  double s = cg_sum_partials(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    st->rr = s;
    st->iters += 1;
    hist.rr(b)[st->iters] = s;
    if (!isfinite(s)) cg_stop(st, DDG_ERR_BREAKDOWN);
    else if (s <= st->tol2) cg_stop(st, DDG_OK);
    else if (st->iters >= st->max_iter) cg_stop(st, DDG_ERR_NO_CONVERGENCE);
  }
}

// partial a.b
__device__ inline void d_dot(const SegMap& m, int g, const double* __restrict__ a, const double* __restrict__ b,
                             double* __restrict__ part) {
  __shared__ double red[kCgThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) acc += a[i] * b[i];
  double s = cg_block_sum(acc, red);
  if (threadIdx.x == 0) part[g] = s;
}

// partials r.z and z.q in one pass (Polak-Ribiere direction update)
__device__ inline void d_dot2(const SegMap& m, int g, const double* __restrict__ r, const double* __restrict__ z,
                              const double* __restrict__ q, double* __restrict__ part, double* __restrict__ part2) {
  __shared__ double red[kCgThreads / 64];
  double a1 = 0.0, a2 = 0.0;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) {
    const double zi = z[i];
    a1 += r[i] * zi;
    a2 += zi * q[i];
  }
  double s1 = cg_block_sum(a1, red);
  double s2 = cg_block_sum(a2, red);
  if (threadIdx.x == 0) {
    part[g] = s1;
    part2[g] = s2;
  }
}

// p = z + beta p
__device__ inline void d_xpby(const CgState* st, const SegMap& m, int g, const double* __restrict__ z,
                              double* __restrict__ p) {
  const double b = st->beta;
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) p[i] = z[i] + b * p[i];
}

// e = 0 on the rows of chunk g
__device__ inline void d_zero(const SegMap& m, int g, double* __restrict__ e) {
  const int64_t hi = m.hi[g];
  for (int64_t i = cg_first(m, g); i < hi; i += kCgThreads) e[i] = 0.0;
}

}  // namespace ddg
