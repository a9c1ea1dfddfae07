// CG kernels (Sections 1 and 7: CG from x0 = 0, stop at ||r|| <= rtol ||f||).
// All vectors float64.  A handle may hold several independent systems (a
// batch); each has its own CG state and its own scalars, and its rows form one
// contiguous segment of every vector.  Reductions are two-stage and
// fixed-order: workgroup g covers a contiguous row range of one system and
// writes one partial (wave butterfly, then waves in order); a scalar kernel
// with one workgroup per system sums that system's partials in a fixed tree,
// so results are bitwise reproducible.  Every kernel first reads its system's
// CG state and returns when that system has stopped, so whole iterations can
// be enqueued ahead of the host's convergence checks and converged systems of
// a batch drop out of every launch.
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

struct SegMap {
  const int32_t* seg;   // system of each workgroup
  const int64_t* lo;    // first row
  const int64_t* hi;    // end row
  const int32_t* ptr;   // nb+1: partials of system b are [ptr[b], ptr[b+1])
};

// Row-dot kernels take L lanes per CSR row (row_dot_l): a workgroup covers
// kThreads / L rows per pass and lane 0 of each group stores the row's result.
// With diagonal storage (D.diag non-null, L = 1) the rows come from the diagonals.
template <int L>
__global__ void k_spmv(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                       const double* __restrict__ v, DiaView D, const double* __restrict__ x,
                       double* __restrict__ y, int64_t n) {
  const int j = threadIdx.x & (L - 1);
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x / L;
  if (L == 1 && D.diag) {
    for (; i < n; i += stride) y[i] = dia_row_dot(D, D.sys[dia_system_of(D, i)], x, i);
    return;
  }
  for (; i < n; i += stride) {
    const double s = row_dot_l<L>(rp, ci, v, x, i, j);
    if (j == 0) y[i] = s;
  }
}

// Diagonal storage from the CSR values: row g's diagonal entry and its entries at
// g + o_d (up was cleared first, so absent entries stay zero).
__global__ void k_dia_fill(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ v, DiaView D, double* __restrict__ diag,
                           double* __restrict__ up) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < D.n; g += stride) {
    const DiaSys& s = D.sys[dia_system_of(D, g)];
    for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
      const int64_t c = ci[t];
      if (c == g) diag[g] = v[t];
      if (c <= g) continue;
      for (int d = 0; d < s.nd; ++d)
        if (c - g == s.off[d]) up[(int64_t)d * D.n + g] = v[t];
    }
  }
}

// Counts lower entries A[g, g - o] whose bits differ from the stored upper entry
// A[g - o, g] (the diagonal storage then does not represent A exactly).
__global__ void k_dia_check(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, DiaView D, int32_t* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < D.n; g += stride) {
    const DiaSys& s = D.sys[dia_system_of(D, g)];
    for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
      const int64_t c = ci[t];
      if (c >= g) break;
      for (int d = 0; d < s.nd; ++d)
        if (g - c == s.off[d] && __double_as_longlong(D.up[(int64_t)d * D.n + c]) != __double_as_longlong(v[t]))
          atomicAdd(bad, 1);
    }
  }
}

// x = 0, r = f, partial f.f
__global__ void k_cg_init(SegMap m, const double* __restrict__ f, double* __restrict__ x,
                          double* __restrict__ r, double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
    double fi = f[i];
    x[i] = 0.0;
    r[i] = fi;
    acc += fi * fi;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ inline uint64_t device_clock() { return wall_clock64(); }

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

__global__ void k_cg_init_scalar(CgState* stb, SegMap m, const double* __restrict__ part, double rtol,
                                 int max_iter, Hist hist) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.x;
  CgState* st = stb + b;
  double s = sum_partials<kThreads>(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
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
__global__ void k_copy_dot(const CgState* stb, SegMap m, const double* __restrict__ r,
                           const double* __restrict__ z, double* __restrict__ p,
                           double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
    double zi = z[i];
    p[i] = zi;
    acc += r[i] * zi;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ inline void stop(CgState* st, int32_t status) {
  st->status = status;
  st->done = 1;
  st->t_done = device_clock();
}

// rho' = r^T z from the partials; beta = rho' / rho (Fletcher-Reeves), or with
// the z^T q partials (part2 non-null) the Polak-Ribiere value
// z^T (r - r_prev) / rho = -alpha z^T q / rho, since r - r_prev = -alpha q.
__global__ void k_rho_scalar(CgState* stb, SegMap m, const double* __restrict__ part,
                             const double* __restrict__ part2, int first, Hist hist) {
  const int b = blockIdx.x;
  CgState* st = stb + b;
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  double zq = 0.0;
  if (part2) zq = sum_partials<kThreads>(part2 + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    if (!(s > 0.0) || !isfinite(s)) {
      stop(st, DDG_ERR_BREAKDOWN);
      return;
    }
    if (first) {
      st->rho = s;
    } else {
      const double beta = part2 ? -st->alpha * zq / st->rho : s / st->rho;
      if (!isfinite(beta)) {
        stop(st, DDG_ERR_BREAKDOWN);
        return;
      }
      st->beta = beta;
      st->rho = s;
      hist.beta(b)[st->iters - 1] = beta;
    }
  }
}

// q = A p, partial p.q
template <int L>
__global__ void k_spmv_dot(const CgState* stb, SegMap m, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v, DiaView D,
                           const double* __restrict__ p, double* __restrict__ q,
                           double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  const int j = threadIdx.x & (L - 1);
  if (L == 1 && D.diag) {
    const DiaSys& sy = D.sys[m.seg[blockIdx.x]];
    for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
      const double qi = dia_row_dot(D, sy, p, i);
      q[i] = qi;
      acc += p[i] * qi;
    }
  } else {
    for (int64_t i = m.lo[blockIdx.x] + threadIdx.x / L; i < hi; i += kThreads / L) {
      const double qi = row_dot_l<L>(rp, ci, v, p, i, j);
      if (j == 0) {
        q[i] = qi;
        acc += p[i] * qi;
      }
    }
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_alpha_scalar(CgState* stb, SegMap m, const double* __restrict__ part, Hist hist) {
  const int b = blockIdx.x;
  CgState* st = stb + b;
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    st->pq = s;
    if (!(s > 0.0) || !isfinite(s)) {
      stop(st, DDG_ERR_BREAKDOWN);
      return;
    }
    st->alpha = st->rho / s;
    hist.alpha(b)[st->iters] = st->alpha;
  }
}

// x += alpha p, r -= alpha q, partial r.r
__global__ void k_axpy2_dot(const CgState* stb, SegMap m, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            double* __restrict__ part) {
  const CgState* st = stb + m.seg[blockIdx.x];
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  const double a = st->alpha;
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
    x[i] += a * p[i];
    double ri = r[i] - a * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_conv_scalar(CgState* stb, SegMap m, const double* __restrict__ part, Hist hist) {
  const int b = blockIdx.x;
  CgState* st = stb + b;
  if (st->done) return;
  __shared__ double red[kThreads / 64];
  double s = sum_partials<kThreads>(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) {
    st->rr = s;
    st->iters += 1;
    hist.rr(b)[st->iters] = s;
    if (!isfinite(s)) stop(st, DDG_ERR_BREAKDOWN);
    else if (s <= st->tol2) stop(st, DDG_OK);
    else if (st->iters >= st->max_iter) stop(st, DDG_ERR_NO_CONVERGENCE);
  }
}

// partial r.z (after the preconditioner)
__global__ void k_dot(const CgState* stb, SegMap m, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) acc += a[i] * b[i];
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// partials r.z and z.q in one pass (Polak-Ribiere direction update)
__global__ void k_dot2(const CgState* stb, SegMap m, const double* __restrict__ r, const double* __restrict__ z,
                       const double* __restrict__ q, double* __restrict__ part, double* __restrict__ part2) {
  if (stb[m.seg[blockIdx.x]].done) return;
  __shared__ double red[kThreads / 64];
  double a1 = 0.0, a2 = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
    const double zi = z[i];
    a1 += r[i] * zi;
    a2 += zi * q[i];
  }
  double s1 = block_sum<kThreads>(a1, red);
  double s2 = block_sum<kThreads>(a2, red);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part2[blockIdx.x] = s2;
  }
}

// p = z + beta p
__global__ void k_xpby(const CgState* stb, SegMap m, const double* __restrict__ z, double* __restrict__ p) {
  const CgState* st = stb + m.seg[blockIdx.x];
  if (st->done) return;
  const double b = st->beta;
  const int64_t hi = m.hi[blockIdx.x];
  for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) p[i] = z[i] + b * p[i];
}

// partial ||f - A x||^2 (always runs)
template <int L>
__global__ void k_resid_dot(SegMap m, const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ v, DiaView D, const double* __restrict__ f,
                            const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  double acc = 0.0;
  const int64_t hi = m.hi[blockIdx.x];
  const int j = threadIdx.x & (L - 1);
  if (L == 1 && D.diag) {
    const DiaSys& sy = D.sys[m.seg[blockIdx.x]];
    for (int64_t i = m.lo[blockIdx.x] + threadIdx.x; i < hi; i += kThreads) {
      const double d = f[i] - dia_row_dot(D, sy, x, i);
      acc += d * d;
    }
  } else {
    for (int64_t i = m.lo[blockIdx.x] + threadIdx.x / L; i < hi; i += kThreads / L) {
      const double d = f[i] - row_dot_l<L>(rp, ci, v, x, i, j);
      if (j == 0) acc += d * d;
    }
  }
  double s = block_sum<kThreads>(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_true_scalar(CgState* stb, SegMap m, const double* __restrict__ part) {
  __shared__ double red[kThreads / 64];
  const int b = blockIdx.x;
  double s = sum_partials<kThreads>(part + m.ptr[b], m.ptr[b + 1] - m.ptr[b], red);
  if (threadIdx.x == 0) stb[b].true_rr = s;
}

int grid_for(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, 4096));
}

SegMap segmap(const Handle& h) {
  return SegMap{h.wg_seg.as<int32_t>(), h.wg_lo.as<int64_t>(), h.wg_hi.as<int64_t>(), h.seg_wg_ptr_d.as<int32_t>()};
}

Hist history(const Handle& h) { return Hist{h.hist.as<double>(), (int64_t)h.opt.max_iter + 1}; }

}  // namespace

// Row ranges of the reduction workgroups: each system is cut into at most 1024
// contiguous chunks (a multiple of 256 rows) of at least 2048 rows, or 2048 / L
// rows (but 256 at least) when the row dots take L lanes per row.
void build_cg_map(Handle& h, hipStream_t s) {
  std::vector<int32_t> seg;
  std::vector<int64_t> lo, hi;
  h.seg_wg_ptr.assign(h.nb + 1, 0);
  const int64_t min_chunk = std::max(256, 2048 / std::max(1, h.lpr));
  for (int32_t b = 0; b < h.nb; ++b) {
    const int64_t a0 = h.seg_off[b], a1 = h.seg_off[b + 1], nb = a1 - a0;
    int64_t chunk = std::max<int64_t>(min_chunk, (nb + 1023) / 1024);
    chunk = (chunk + kThreads - 1) / kThreads * kThreads;
    int64_t cnt = std::max<int64_t>(1, (nb + chunk - 1) / chunk);
    for (int64_t c = 0; c < cnt; ++c) {
      seg.push_back(b);
      lo.push_back(a0 + std::min(nb, c * chunk));
      hi.push_back(a0 + std::min(nb, (c + 1) * chunk));
    }
    h.seg_wg_ptr[b + 1] = (int32_t)seg.size();
  }
  h.n_partials = (int32_t)seg.size();
  h.wg_seg.upload(seg, s);
  h.wg_lo.upload(lo, s);
  h.wg_hi.upload(hi, s);
  h.seg_wg_ptr_d.upload(h.seg_wg_ptr, s);
  // two partial arrays: the Polak-Ribiere update reduces r.z and z.q together
  h.part_sums.alloc((size_t)2 * h.n_partials * sizeof(double));
  h.hist.alloc((size_t)h.nb * 3 * ((size_t)h.opt.max_iter + 1) * sizeof(double));
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kThreads), 0, s, x, v, n);
}

void launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(grid_for(n)), dim3(kThreads), 0, s, dst, src, n);
}

void launch_spmv(const Handle& h, const double* x, double* y, hipStream_t s) {
  with_lanes(h.lpr, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    hipLaunchKernelGGL(k_spmv<L>, dim3(grid_for(h.S.n * L)), dim3(kThreads), 0, s, h.rowptr.as<int64_t>(),
                       h.col.as<int32_t>(), h.val.as<double>(), dia_view(h), x, y, h.S.n);
  });
}

void launch_dia_refresh(Handle& h, hipStream_t s) {
  if (!h.dia_possible) return;
  DiaView D{};
  D.diag = h.dia_diag.as<double>();
  D.up = h.dia_up.as<double>();
  D.sys = h.dia_sys.as<DiaSys>();
  D.n = h.S.n;
  D.nb = h.nb;
  launch_fill(h.dia_up.as<double>(), 0.0, (int64_t)h.dia_nd * h.S.n, s);
  hipLaunchKernelGGL(k_dia_fill, dim3(grid_for(h.S.n)), dim3(kThreads), 0, s, h.rowptr.as<int64_t>(),
                     h.col.as<int32_t>(), h.val.as<double>(), D, h.dia_diag.as<double>(), h.dia_up.as<double>());
  hipLaunchKernelGGL(k_dia_check, dim3(grid_for(h.S.n)), dim3(kThreads), 0, s, h.rowptr.as<int64_t>(),
                     h.col.as<int32_t>(), h.val.as<double>(), D, h.err_flag.as<int32_t>() + 4);
  DDG_HIP(hipGetLastError());
}

void launch_cg_init(Handle& h, const double* f, double* x, hipStream_t s) {
  const SegMap m = segmap(h);
  hipLaunchKernelGGL(k_cg_init, dim3(h.n_partials), dim3(kThreads), 0, s, m, f, x, h.r.as<double>(),
                     h.part_sums.as<double>());
  hipLaunchKernelGGL(k_cg_init_scalar, dim3(h.nb), dim3(kThreads), 0, s, h.cstate.as<CgState>(), m,
                     h.part_sums.as<double>(), h.opt.rtol, h.opt.max_iter, history(h));
}

void launch_cg_start(Handle& h, hipStream_t s) {
  const SegMap m = segmap(h);
  CgState* st = h.cstate.as<CgState>();
  hipLaunchKernelGGL(k_copy_dot, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, h.r.as<double>(),
                     h.z.as<double>(), h.p.as<double>(), h.part_sums.as<double>());
  hipLaunchKernelGGL(k_rho_scalar, dim3(h.nb), dim3(kThreads), 0, s, st, m, h.part_sums.as<double>(),
                     (const double*)nullptr, 1, history(h));
}

void launch_cg_step_a(Handle& h, double* x, hipStream_t s) {
  const SegMap m = segmap(h);
  CgState* st = h.cstate.as<CgState>();
  with_lanes(h.lpr, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    hipLaunchKernelGGL(k_spmv_dot<L>, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, h.rowptr.as<int64_t>(),
                       h.col.as<int32_t>(), h.val.as<double>(), dia_view(h), h.p.as<double>(), h.q.as<double>(),
                       h.part_sums.as<double>());
  });
  hipLaunchKernelGGL(k_alpha_scalar, dim3(h.nb), dim3(kThreads), 0, s, st, m, h.part_sums.as<double>(), history(h));
  hipLaunchKernelGGL(k_axpy2_dot, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, x, h.r.as<double>(),
                     h.p.as<double>(), h.q.as<double>(), h.part_sums.as<double>());
  hipLaunchKernelGGL(k_conv_scalar, dim3(h.nb), dim3(kThreads), 0, s, st, m, h.part_sums.as<double>(), history(h));
}

void launch_cg_step_b(Handle& h, hipStream_t s) {
  const SegMap m = segmap(h);
  CgState* st = h.cstate.as<CgState>();
  double* part = h.part_sums.as<double>();
  double* part2 = nullptr;
  if (h.opt.cg_variant == DDG_CG_POLAK_RIBIERE) {
    part2 = part + h.n_partials;
    hipLaunchKernelGGL(k_dot2, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, h.r.as<double>(), h.z.as<double>(),
                       h.q.as<double>(), part, part2);
  } else {
    hipLaunchKernelGGL(k_dot, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, h.r.as<double>(), h.z.as<double>(),
                       part);
  }
  hipLaunchKernelGGL(k_rho_scalar, dim3(h.nb), dim3(kThreads), 0, s, st, m, part, (const double*)part2, 0,
                     history(h));
  hipLaunchKernelGGL(k_xpby, dim3(h.n_partials), dim3(kThreads), 0, s, st, m, h.z.as<double>(), h.p.as<double>());
}

void launch_true_residual(Handle& h, const double* f, const double* x, hipStream_t s) {
  const SegMap m = segmap(h);
  with_lanes(h.lpr, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    hipLaunchKernelGGL(k_resid_dot<L>, dim3(h.n_partials), dim3(kThreads), 0, s, m, h.rowptr.as<int64_t>(),
                       h.col.as<int32_t>(), h.val.as<double>(), dia_view(h), f, x, h.part_sums.as<double>());
  });
  hipLaunchKernelGGL(k_true_scalar, dim3(h.nb), dim3(kThreads), 0, s, h.cstate.as<CgState>(), m,
                     h.part_sums.as<double>());
}

}  // namespace ddg
