// CG kernels (Sections 1 and 7: CG from x0 = 0, stop at ||r|| <= rtol ||f||).
// All vectors float64.  Reductions are two-stage and fixed-order: each
// workgroup writes one partial (wave butterfly, then waves in order) and a
// one-workgroup scalar kernel sums the partials in a fixed tree, so results
// are bitwise reproducible.  Every kernel first reads the device CG state and
// returns when the solve has stopped, so whole iterations can be enqueued
// ahead of the host's convergence checks.
#include "common.hpp"
#include "device_util.hpp"

namespace ddg {

namespace {

constexpr int kThreads = 256;

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) x[i] = v;
}

__global__ void k_copy(double* __restrict__ d, const double* __restrict__ s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) d[i] = s[i];
}

__device__ inline double row_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ v, const double* __restrict__ x,
                                 int64_t g) {
  double s = 0.0;
  for (int64_t t = rp[g]; t < rp[g + 1]; ++t) s += v[t] * x[ci[t]];
  return s;
}

__global__ void k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ v, const double* __restrict__ x,
                       double* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] = row_dot(rp, ci, v, x, i);
}

// x = 0, r = f, partial f.f
__global__ void k_cg_init(const double* __restrict__ f, double* __restrict__ x,
                          double* __restrict__ r, double* __restrict__ part, int64_t n) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double fi = f[i];
    x[i] = 0.0;
    r[i] = fi;
    acc += fi * fi;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_cg_init_scalar(CgState* st, const double* __restrict__ part, int np, double rtol,
                                 int max_iter) {
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part, np, red);
  if (threadIdx.x == 0) {
    st->iters = 0;
    st->max_iter = max_iter;
    st->status = DDG_OK;
    st->done = 0;
    st->fnorm = sqrt(s);
    st->rr = s;
    st->tol2 = rtol * rtol * s;
    st->rho = st->alpha = st->beta = st->pq = 0.0;
    st->true_rr = 0.0;
    if (!isfinite(s)) {
      st->status = DDG_ERR_INVALID_ARG;
      st->done = 1;
    } else if (s == 0.0) {
      st->done = 1;
    }
  }
}

// p = z, partial r.z
__global__ void k_copy_dot(const CgState* st, const double* __restrict__ r,
                           const double* __restrict__ z, double* __restrict__ p,
                           double* __restrict__ part, int64_t n) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double zi = z[i];
    p[i] = zi;
    acc += r[i] * zi;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_rho_scalar(CgState* st, const double* __restrict__ part, int np, int first) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part, np, red);
  if (threadIdx.x == 0) {
    if (!(s > 0.0) || !isfinite(s)) {
      st->status = DDG_ERR_BREAKDOWN;
      st->done = 1;
      return;
    }
    if (first) {
      st->rho = s;
    } else {
      st->beta = s / st->rho;
      st->rho = s;
    }
  }
}

// q = A p, partial p.q
__global__ void k_spmv_dot(const CgState* st, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v,
                           const double* __restrict__ p, double* __restrict__ q,
                           double* __restrict__ part, int64_t n) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double qi = row_dot(rp, ci, v, p, i);
    q[i] = qi;
    acc += p[i] * qi;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_alpha_scalar(CgState* st, const double* __restrict__ part, int np) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part, np, red);
  if (threadIdx.x == 0) {
    st->pq = s;
    if (!(s > 0.0) || !isfinite(s)) {
      st->status = DDG_ERR_BREAKDOWN;
      st->done = 1;
      return;
    }
    st->alpha = st->rho / s;
  }
}

// x += alpha p, r -= alpha q, partial r.r
__global__ void k_axpy2_dot(const CgState* st, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            double* __restrict__ part, int64_t n) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  const double a = st->alpha;
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    x[i] += a * p[i];
    double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_conv_scalar(CgState* st, const double* __restrict__ part, int np) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part, np, red);
  if (threadIdx.x == 0) {
    st->rr = s;
    st->iters += 1;
    if (!isfinite(s)) {
      st->status = DDG_ERR_BREAKDOWN;
      st->done = 1;
    } else if (s <= st->tol2) {
      st->status = DDG_OK;
      st->done = 1;
    } else if (st->iters >= st->max_iter) {
      st->status = DDG_ERR_NO_CONVERGENCE;
      st->done = 1;
    }
  }
}

// partial r.z (after the preconditioner)
__global__ void k_dot(const CgState* st, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ part, int64_t n) {
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    acc += a[i] * b[i];
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p
__global__ void k_xpby(const CgState* st, const double* __restrict__ z, double* __restrict__ p,
                       int64_t n) {
  if (st->done) return;
  const double b = st->beta;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = z[i] + b * p[i];
}

// partial ||f - A x||^2 (always runs)
__global__ void k_resid_dot(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, const double* __restrict__ f,
                            const double* __restrict__ x, double* __restrict__ part, int64_t n) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double d = f[i] - row_dot(rp, ci, v, x, i);
    acc += d * d;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_true_scalar(CgState* st, const double* __restrict__ part, int np) {
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part, np, red);
  if (threadIdx.x == 0) st->true_rr = s;
}

int grid_for(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

}  // namespace

int32_t cg_partials_count(int64_t n) {
  int64_t g = (n + kThreads * 4 - 1) / (kThreads * 4);
  return (int32_t)std::max<int64_t>(1, std::min<int64_t>(g, 1024));
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, x, v, n);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n);
}

void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_spmv, dim3(grid_for(h.S.n)), dim3(kThreads), 0, s, h.rowptr.as<int64_t>(),
                     h.col.as<int32_t>(), h.val.as<double>(), x, y, h.S.n);
}

void launch_cg_init(Handle& h, const double* f, double* x, hipStream_t s) {
  int np = h.n_partials;
  hipLaunchKernelGGL(k_cg_init, dim3(np), dim3(kThreads), 0, s, f, x, h.r.as<double>(),
                     h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_cg_init_scalar, dim3(1), dim3(kThreads), 0, s, h.cstate.as<CgState>(),
                     h.part_sums.as<double>(), np, h.opt.rtol, h.opt.max_iter);
}

void launch_cg_start(Handle& h, hipStream_t s) {
  int np = h.n_partials;
  CgState* st = h.cstate.as<CgState>();
  hipLaunchKernelGGL(k_copy_dot, dim3(np), dim3(kThreads), 0, s, st, h.r.as<double>(),
                     h.z.as<double>(), h.p.as<double>(), h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_rho_scalar, dim3(1), dim3(kThreads), 0, s, st, h.part_sums.as<double>(), np, 1);
}

void launch_cg_step_a(Handle& h, double* x, hipStream_t s) {
  int np = h.n_partials;
  CgState* st = h.cstate.as<CgState>();
  hipLaunchKernelGGL(k_spmv_dot, dim3(np), dim3(kThreads), 0, s, st, h.rowptr.as<int64_t>(),
                     h.col.as<int32_t>(), h.val.as<double>(), h.p.as<double>(), h.q.as<double>(),
                     h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_alpha_scalar, dim3(1), dim3(kThreads), 0, s, st, h.part_sums.as<double>(), np);
  hipLaunchKernelGGL(k_axpy2_dot, dim3(np), dim3(kThreads), 0, s, st, x, h.r.as<double>(),
                     h.p.as<double>(), h.q.as<double>(), h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_conv_scalar, dim3(1), dim3(kThreads), 0, s, st, h.part_sums.as<double>(), np);
}

void launch_cg_step_b(Handle& h, hipStream_t s) {
  int np = h.n_partials;
  CgState* st = h.cstate.as<CgState>();
  hipLaunchKernelGGL(k_dot, dim3(np), dim3(kThreads), 0, s, st, h.r.as<double>(), h.z.as<double>(),
                     h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_rho_scalar, dim3(1), dim3(kThreads), 0, s, st, h.part_sums.as<double>(), np, 0);
  hipLaunchKernelGGL(k_xpby, dim3(grid_for(h.S.n)), dim3(kThreads), 0, s, st, h.z.as<double>(),
                     h.p.as<double>(), h.S.n);
}

void launch_true_residual(Handle& h, const double* f, const double* x, hipStream_t s) {
  int np = h.n_partials;
  hipLaunchKernelGGL(k_resid_dot, dim3(np), dim3(kThreads), 0, s, h.rowptr.as<int64_t>(),
                     h.col.as<int32_t>(), h.val.as<double>(), f, x, h.part_sums.as<double>(), h.S.n);
  hipLaunchKernelGGL(k_true_scalar, dim3(1), dim3(kThreads), 0, s, h.cstate.as<CgState>(),
                     h.part_sums.as<double>(), np);
}

}  // namespace ddg
