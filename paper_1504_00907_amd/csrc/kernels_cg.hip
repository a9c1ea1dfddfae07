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
#include "cg_device.hpp"

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

// One workgroup per row chunk (SegMap) or per system; the bodies are in cg_device.hpp.
__global__ void k_cg_init(SegMap m, const double* __restrict__ f, double* __restrict__ x,
                          double* __restrict__ r, double* __restrict__ part) {
  d_cg_init(m, blockIdx.x, f, x, r, part);
}

__global__ void k_cg_init_scalar(CgState* stb, SegMap m, const double* __restrict__ part, double rtol,
                                 int max_iter, Hist hist) {
  d_cg_init_scalar(stb, m, blockIdx.x, part, rtol, max_iter, hist);
}

__global__ void k_copy_dot(const CgState* stb, SegMap m, const double* __restrict__ r,
                           const double* __restrict__ z, double* __restrict__ p,
                           double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  d_copy_dot(m, blockIdx.x, r, z, p, part);
}

__global__ void k_rho_scalar(CgState* stb, SegMap m, const double* __restrict__ part,
                             const double* __restrict__ part2, int first, Hist hist) {
  if (stb[blockIdx.x].done) return;
  d_rho_scalar(stb, m, blockIdx.x, part, part2, first, hist);
}

template <int L>
__global__ void k_spmv_dot(const CgState* stb, SegMap m, const int64_t* __restrict__ rp,
                           const int32_t* __restrict__ ci, const double* __restrict__ v, DiaView D,
                           const double* __restrict__ p, double* __restrict__ q,
                           double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  d_spmv_dot<L>(m, blockIdx.x, rp, ci, v, D, p, q, part);
}

__global__ void k_alpha_scalar(CgState* stb, SegMap m, const double* __restrict__ part, Hist hist) {
  if (stb[blockIdx.x].done) return;
  d_alpha_scalar(stb, m, blockIdx.x, part, hist);
}

__global__ void k_axpy2_dot(const CgState* stb, SegMap m, double* __restrict__ x, double* __restrict__ r,
                            const double* __restrict__ p, const double* __restrict__ q,
                            double* __restrict__ part) {
  const CgState* st = stb + m.seg[blockIdx.x];
  if (st->done) return;
  d_axpy2_dot(st, m, blockIdx.x, x, r, p, q, part);
}

__global__ void k_conv_scalar(CgState* stb, SegMap m, const double* __restrict__ part, Hist hist) {
  if (stb[blockIdx.x].done) return;
  d_conv_scalar(stb, m, blockIdx.x, part, hist);
}

__global__ void k_dot(const CgState* stb, SegMap m, const double* __restrict__ a, const double* __restrict__ b,
                      double* __restrict__ part) {
  if (stb[m.seg[blockIdx.x]].done) return;
  d_dot(m, blockIdx.x, a, b, part);
}

__global__ void k_dot2(const CgState* stb, SegMap m, const double* __restrict__ r, const double* __restrict__ z,
                       const double* __restrict__ q, double* __restrict__ part, double* __restrict__ part2) {
  if (stb[m.seg[blockIdx.x]].done) return;
  d_dot2(m, blockIdx.x, r, z, q, part, part2);
}

__global__ void k_xpby(const CgState* stb, SegMap m, const double* __restrict__ z, double* __restrict__ p) {
  const CgState* st = stb + m.seg[blockIdx.x];
  if (st->done) return;
  d_xpby(st, m, blockIdx.x, z, p);
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
