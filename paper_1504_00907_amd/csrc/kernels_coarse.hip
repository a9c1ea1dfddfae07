// Coarse correction of the two-level preconditioner (Section 4 coarse problem,
// Section 6 multiplicative combination):
//     e += R0^T A0^{-1} R0 (r - A e)
// R0^T = blockdiag(Q_i) with Q_i the orthonormal basis of subdomain i, so
//   b0[off_i + m] = sum_{g in Omega_i} Q[g, m] (r - A e)_g        (restrict)
//   y = A0^{-1} b0                                                  (tiled symmetric GEMV)
//   e_g += sum_m Q[g, m] y[off_{part g} + m]                        (prolong)
// (restriction and prolongation read Q in the own-row layout q_own_at)
// A0^{-1} is the explicit float64 inverse computed at setup; it is stored as
// lower 64 x 64 tiles and applied with one wave per tile, writing fixed
// per-tile partials that a second kernel sums in a fixed order.  With several
// independent systems A0 is block diagonal: system b owns the padded coarse
// rows [cblk_off[b], cblk_off[b+1]) and the tiles [tile_base[b], tile_base[b+1])
// of its own inverse; kernels skip the work of systems that have stopped.
#include "coarse_device.hpp"

namespace ddg {

namespace {

template <int L, int KM>
__global__ void __launch_bounds__(kRThreads) k_coarse_restrict(
    const CgState* st, const int32_t* __restrict__ sub_inst, const int64_t* __restrict__ own_ptr,
    const int32_t* __restrict__ own_idx, const int32_t* __restrict__ kcnt, const double* __restrict__ Qo, int kq,
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ val,
    DiaView D, const double* __restrict__ r, const double* __restrict__ e, int rch, double* __restrict__ rpart) {
  const int i = blockIdx.y, c = blockIdx.x;
  if (st && st[sub_inst[i]].done) return;
  d_coarse_restrict<L, KM>(i, c, gridDim.x, sub_inst, own_ptr, own_idx, kcnt, Qo, kq, rp, ci, val, D, r, e, rch, rpart);
}

// b0[koff[i] + m] = sum over the nch chunks of subdomain i, in chunk order
__global__ void k_coarse_restrict_sum(const CgState* st, const int32_t* __restrict__ sub_inst,
                                      const int32_t* __restrict__ kcnt, const int64_t* __restrict__ koff,
                                      const double* __restrict__ rpart, int nch, int n_parts, int KM,
                                      double* __restrict__ b0) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(id / KM), m = (int)(id % KM);
  if (i >= n_parts) return;
  if (st && st[sub_inst[i]].done) return;
  d_coarse_restrict_sum_entry(i, m, kcnt, koff, rpart, nch, KM, b0);
}

// one wave per 64x64 float64 tile: row and column partials into per-tile slots
__global__ void __launch_bounds__(256) k_coarse_symv(const CgState* st, const int32_t* __restrict__ tile_inst,
                                                     const int64_t* __restrict__ tile_base,
                                                     const int64_t* __restrict__ cblk_off,
                                                     const double* __restrict__ tiles, int64_t ntiles,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ rowpart,
                                                     double* __restrict__ colpart) {
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const int b = tile_inst[t];
  if (st && st[b].done) return;
  d_coarse_symv_tile(t, b, tile_base, cblk_off, tiles, x, rowpart, colpart);
}

// y over the padded coarse rows; trow_inst gives the system of each 64-row tile row
__global__ void k_coarse_sum(const CgState* st, const int32_t* __restrict__ trow_inst,
                             const int64_t* __restrict__ tile_base, const int64_t* __restrict__ cblk_off,
                             const double* __restrict__ rowpart, const double* __restrict__ colpart,
                             int64_t nc_pad, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc_pad) return;
  const int b = trow_inst[row / 64];
  if (st && st[b].done) return;
  d_coarse_sum_row(row, b, tile_base, cblk_off, rowpart, colpart, y);
}

// one thread per row, in the own-row order (the basis reads are contiguous)
// The basis in the own-row layout (q_own_at) and each row's position in the
// own-row order, from the node-major basis of the setup.
__global__ void k_q_own(const int32_t* __restrict__ own_idx, const double* __restrict__ Q, int64_t n, int k,
                        double* __restrict__ Qo, int32_t* __restrict__ qpos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int g = own_idx[t];
  qpos[g] = (int32_t)t;
  for (int m = 0; m < k; ++m) Qo[q_own_at(t, m, k)] = Q[(int64_t)g * k + m];
}

template <int KM>
__global__ void __launch_bounds__(256) k_coarse_prolong(const CgState* st, const int32_t* __restrict__ sub_inst,
                                 const int32_t* __restrict__ part, const int32_t* __restrict__ own_idx,
                                 const int32_t* __restrict__ kcnt, const int64_t* __restrict__ koff,
                                 const double* __restrict__ Qo, int kq, const double* __restrict__ y,
                                 double* __restrict__ e, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  d_coarse_prolong_row<KM>(own_idx[t], t, st, sub_inst, part, kcnt, koff, Qo, kq, y, e);
}

// F0[koff[i] + j, c] = sum over the own rows g of subdomain i of Q[g, j] F[g, c]
// (F0 = R0 F); one workgroup per subdomain, one thread per (j, c), rows in order.
__global__ void k_restrict_columns(const int64_t* __restrict__ own_ptr, const int32_t* __restrict__ own_idx,
                                   const int32_t* __restrict__ kcnt, const int64_t* __restrict__ koff,
                                   const double* __restrict__ Q, int kq, const double* __restrict__ F, int64_t n,
                                   int64_t ld0, double* __restrict__ F0) {
  const int i = blockIdx.x;
  const int ki = kcnt[i];
  for (int t = threadIdx.x; t < ki * kq; t += blockDim.x) {
    const int j = t % ki, c = t / ki;
    double s = 0.0;
    for (int64_t u = own_ptr[i]; u < own_ptr[i + 1]; ++u) {
      const int g = own_idx[u];
      s += Q[(int64_t)g * kq + j] * F[(int64_t)c * n + g];
    }
    F0[(int64_t)c * ld0 + koff[i] + j] = s;
  }
}

// t[row] = b[row] - (A0 y)[row] over the padded coarse rows (one wave per row, the
// columns of the row's system in lane order then a butterfly); 0 on padding rows
__global__ void __launch_bounds__(256) k_a0_resid(const CgState* st, const int32_t* __restrict__ trow_inst,
                                                  const int64_t* __restrict__ cblk_off,
                                                  const int32_t* __restrict__ cblk_n, const int64_t* __restrict__ a0_off,
                                                  const double* __restrict__ A0, const double* __restrict__ b,
                                                  const double* __restrict__ y, int64_t nc_pad,
                                                  double* __restrict__ t) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nc_pad) return;
  const int sys = trow_inst[row / 64];
  if (st && st[sys].done) return;
  const int64_t c0 = cblk_off[sys], N = cblk_n[sys], lr = row - c0;
  double s = 0.0;
  if (lr < N) {
    const double* a = A0 + a0_off[sys] + lr * N;
    for (int64_t j = lane; j < N; j += 64) s += a[j] * y[c0 + j];
  }
  s = wave_sum(s);
  if (lane == 0) t[row] = lr < N ? b[row] - s : 0.0;
}

// y += dy over the padded coarse rows
__global__ void k_coarse_add(const CgState* st, const int32_t* __restrict__ trow_inst, const double* __restrict__ dy,
                             int64_t nc_pad, double* __restrict__ y) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc_pad) return;
  if (st && st[trow_inst[row / 64]].done) return;
  y[row] += dy[row];
}

// v[row] = a fixed pseudo-random value in [-1, 1) (integer hash of the row), 0 on padding rows
__global__ void k_coarse_probe(const int32_t* __restrict__ trow_inst, const int64_t* __restrict__ cblk_off,
                               const int32_t* __restrict__ cblk_n, int64_t nc_pad, double* __restrict__ v) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc_pad) return;
  const int sys = trow_inst[row / 64];
  uint64_t z = (uint64_t)row * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  v[row] = row - cblk_off[sys] < cblk_n[sys] ? (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0 : 0.0;
}

// per system: out[2b] = ||v + u||^2, out[2b+1] = ||v||^2 over its coarse rows (u = -X A0 v)
__global__ void k_coarse_err(const int64_t* __restrict__ cblk_off, const int32_t* __restrict__ cblk_n,
                             const double* __restrict__ v, const double* __restrict__ u, double* __restrict__ out) {
  __shared__ double red[4];
  const int b = blockIdx.x;
  const int64_t c0 = cblk_off[b];
  double a = 0.0, c = 0.0;
  for (int64_t r = threadIdx.x; r < cblk_n[b]; r += 256) {
    const double d = v[c0 + r] + u[c0 + r];
    a += d * d;
    c += v[c0 + r] * v[c0 + r];
  }
  const double sa = block_sum<256>(a, red);
  const double sc = block_sum<256>(c, red);
  if (threadIdx.x == 0) {
    out[2 * b] = sa;
    out[2 * b + 1] = sc;
  }
}

// power-iteration step: v = (v + u) / ||v + u|| per system (u = -X A0 v; out from k_coarse_err)
__global__ void k_coarse_next(const int32_t* __restrict__ trow_inst, const int64_t* __restrict__ cblk_off,
                              const int32_t* __restrict__ cblk_n, int64_t nc_pad, const double* __restrict__ out,
                              const double* __restrict__ u, double* __restrict__ v) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc_pad) return;
  const int sys = trow_inst[row / 64];
  const double nn = out[2 * sys];
  v[row] = row - cblk_off[sys] < cblk_n[sys] && nn > 0.0 ? (v[row] + u[row]) / sqrt(nn) : 0.0;
}

// y = X b with the packed inverse tiles (row and column slots, then the fixed-order sum)
void coarse_symv(Handle& h, const CgState* st, const double* b, double* y, hipStream_t s) {
  double* rowpart = h.ws.cpart;
  double* colpart = rowpart + h.ntiles * 64;
  hipLaunchKernelGGL(k_coarse_symv, dim3((unsigned)((h.ntiles + 3) / 4)), dim3(256), 0, s, st,
                     h.tile_inst.as<int32_t>(), h.tile_base_d.as<int64_t>(), h.cblk_off_d.as<int64_t>(),
                     h.A0inv_t.as<double>(), h.ntiles, b, rowpart, colpart);
  hipLaunchKernelGGL(k_coarse_sum, dim3((unsigned)((h.nc_pad + 255) / 256)), dim3(256), 0, s, st,
                     h.trow_inst.as<int32_t>(), h.tile_base_d.as<int64_t>(), h.cblk_off_d.as<int64_t>(),
                     rowpart, colpart, h.nc_pad, y);
}

// t = b - A0 y on the padded coarse rows
void coarse_resid(Handle& h, const CgState* st, const double* b, const double* y, double* t, hipStream_t s) {
  hipLaunchKernelGGL(k_a0_resid, dim3((unsigned)((h.nc_pad + 3) / 4)), dim3(256), 0, s, st,
                     h.trow_inst.as<int32_t>(), h.cblk_off_d.as<int64_t>(), h.cblk_n_d.as<int32_t>(),
                     h.a0_off_d.as<int64_t>(), h.A0.as<double>(), b, y, h.nc_pad, t);
}

}  // namespace

// Estimate of the spectral radius of I - X A0 (X the explicit coarse inverse), the
// factor by which each refinement step reduces the coarse error: the largest
// ||(I - X A0) v|| / ||v|| over kPowerSteps normalised power-iteration steps from a
// fixed pseudo-random start, worst system.  The steps are enqueued on s with their
// norms copied to pinned host memory; finish_coarse_measure reads them once the
// stream has been synchronised.
constexpr int kPowerSteps = 8;

void launch_coarse_measure(Handle& h, hipStream_t s) {
  if (h.nc == 0 || h.three_level || h.ic) return;
  const size_t nout = (size_t)2 * h.nb * kPowerSteps;
  if (!h.cerr.p) h.cerr.alloc(((size_t)3 * h.nc_pad + nout) * sizeof(double));
  if (!h.h_cerr) DDG_HIP(hipHostMalloc((void**)&h.h_cerr, nout * sizeof(double), hipHostMallocDefault));
  double* v = h.cerr.as<double>();
  double* t = v + h.nc_pad;
  double* u = t + h.nc_pad;
  double* out = u + h.nc_pad;
  const unsigned g = (unsigned)((h.nc_pad + 255) / 256);
  hipLaunchKernelGGL(k_coarse_probe, dim3(g), dim3(256), 0, s, h.trow_inst.as<int32_t>(), h.cblk_off_d.as<int64_t>(),
                     h.cblk_n_d.as<int32_t>(), h.nc_pad, v);
  PrecondWs keep = h.ws;
  if (!h.ws.cpart) h.ws.cpart = h.cpart.as<double>();
  for (int it = 0; it < kPowerSteps; ++it) {
    double* o = out + (size_t)2 * h.nb * it;
    if (it > 0)
      hipLaunchKernelGGL(k_coarse_next, dim3(g), dim3(256), 0, s, h.trow_inst.as<int32_t>(),
                         h.cblk_off_d.as<int64_t>(), h.cblk_n_d.as<int32_t>(), h.nc_pad, o - 2 * h.nb, u, v);
    launch_fill(u, 0.0, h.nc_pad, s);
    coarse_resid(h, nullptr, u, v, t, s);   // t = 0 - A0 v
    // u = X t = -X A0 v (the handle's own partial slots; no solve is running)
    coarse_symv(h, nullptr, t, u, s);
    hipLaunchKernelGGL(k_coarse_err, dim3((unsigned)h.nb), dim3(256), 0, s, h.cblk_off_d.as<int64_t>(),
                       h.cblk_n_d.as<int32_t>(), v, u, o);
  }
  h.ws = keep;
  DDG_HIP(hipMemcpyAsync(h.h_cerr, out, nout * sizeof(double), hipMemcpyDeviceToHost, s));
  DDG_HIP(hipGetLastError());
}

double finish_coarse_measure(const Handle& h) {
  if (h.nc == 0 || h.three_level || h.ic || !h.h_cerr) return 0.0;
  double worst = 0.0;
  for (int it = 0; it < kPowerSteps; ++it)
    for (int32_t b = 0; b < h.nb; ++b) {
      const double* o = h.h_cerr + (size_t)2 * h.nb * it + 2 * b;
      if (!(o[1] > 0)) continue;
      const double e = std::sqrt(o[0] / o[1]);
      if (!(e <= worst)) worst = e;   // keeps a NaN
    }
  return worst;
}

void launch_q_own(Handle& h, hipStream_t s) {
  const int64_t n = h.S.n;
  h.Qo.alloc((size_t)((n + 63) / 64) * 64 * h.k * sizeof(double));
  h.qpos.alloc((size_t)n * sizeof(int32_t));
  hipLaunchKernelGGL(k_q_own, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, h.own_idx.as<int32_t>(),
                     h.Q.as<double>(), n, h.k, h.Qo.as<double>(), h.qpos.as<int32_t>());
  DDG_HIP(hipGetLastError());
}

void launch_restrict_columns(Handle& h, double* F0, hipStream_t s) {
  launch_fill(F0, 0.0, h.nc_pad * h.k, s);
  hipLaunchKernelGGL(k_restrict_columns, dim3((unsigned)h.S.n_parts), dim3(256), 0, s, h.own_ptr.as<int64_t>(),
                     h.own_idx.as<int32_t>(), h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(), h.Q.as<double>(), h.k,
                     h.F.as<double>(), h.S.n, h.nc_pad, F0);
  DDG_HIP(hipGetLastError());
}

void launch_sweep(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                  const CgState* st, hipStream_t s, bool residual);

template <int KM>
void launch_coarse_k(Handle& h, const double* r, double* e, const CgState* st, hipStream_t s) {
  const Symbolic& S = h.S;
  double* b0 = h.ws.cy;             // padded to whole tiles, zero beyond each block
  double* y = b0 + h.nc_pad;
  const int32_t* sub_inst = h.sub_inst.as<int32_t>();
  DDG_REQUIRE(h.rch * h.lpr == 4 * kRThreads, DDG_ERR_HIP, "internal: restriction chunking");
  with_lanes(h.lpr, [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    hipLaunchKernelGGL((k_coarse_restrict<L, KM>), dim3((unsigned)h.nch, (unsigned)S.n_parts), dim3(kRThreads), 0, s, st,
                       sub_inst, h.own_ptr.as<int64_t>(), h.own_idx.as<int32_t>(), h.kcnt_d.as<int32_t>(),
                       h.Qo.as<double>(), h.k, h.rowptr.as<int64_t>(), h.col.as<int32_t>(), h.val.as<double>(),
                       dia_view(h), r, e, h.rch, h.ws.rpart);
  });
  hipLaunchKernelGGL(k_coarse_restrict_sum, dim3((unsigned)(((int64_t)S.n_parts * KM + 255) / 256)), dim3(256), 0,
                     s, st, sub_inst, h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(), h.ws.rpart, h.nch,
                     S.n_parts, KM, b0);
  if (h.inner) {
    // three levels: y = M0^{-1} b0, one application of the coarse level's two-level
    // preconditioner (its kernels skip work once this handle's system has stopped)
    launch_precond(*h.inner, b0, y, -1, false, s, st);
  } else if (h.ic) {
    // inexact coarse solve: incomplete-Cholesky-preconditioned CG on A0 y = b0
    launch_ic_solve(h, st, b0, y, s);
  } else {
    coarse_symv(h, st, b0, y, s);
    // refinement steps y += X (b0 - A0 y) when the explicit inverse is inaccurate
    for (int32_t j = 0; j < h.coarse_refine; ++j) {
      double* t = h.ws.cref;
      double* dy = t + h.nc_pad;
      coarse_resid(h, st, b0, y, t, s);
      coarse_symv(h, st, t, dy, s);
      hipLaunchKernelGGL(k_coarse_add, dim3((unsigned)((h.nc_pad + 255) / 256)), dim3(256), 0, s, st,
                         h.trow_inst.as<int32_t>(), dy, h.nc_pad, y);
    }
  }
  hipLaunchKernelGGL(k_coarse_prolong<KM>, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, s, st, sub_inst,
                     h.part.as<int32_t>(), h.own_idx.as<int32_t>(), h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(),
                     h.Qo.as<double>(), h.k, y, e, S.n);
  DDG_HIP(hipGetLastError());
}

void launch_coarse(Handle& h, const double* r, double* e, const CgState* st, hipStream_t s) {
  if (h.nc == 0) return;
  DDG_REQUIRE(h.k <= kMaxGen, DDG_ERR_UNSUPPORTED, "at most 80 generating vectors");
  // (the per-thread column arrays sized to the basis: fewer registers and predicated
  // steps for small k; the partial-sum stride stays within the kslots(k) allocation)
  if (h.k <= 16) launch_coarse_k<16>(h, r, e, st, s);
  else if (h.k <= 32) launch_coarse_k<32>(h, r, e, st, s);
  else launch_coarse_k<kMaxGen>(h, r, e, st, s);
}

// Attaches an event pair to the next local-solve dispatch for the scope's lifetime.
struct KernelEvents {
  const Handle& h;
  KernelEvents(const Handle& hh, hipEvent_t a, hipEvent_t b) : h(hh) {
    h.kev0 = a;
    h.kev1 = b;
  }
  ~KernelEvents() { h.kev0 = h.kev1 = nullptr; }
};

// Local residual of one colour, then its local solves; when profiling, the local-solve
// dispatch carries an event pair that records its own start and end.
static void sweep_profiled(Handle& h, int c, const double* r, double* e, bool ez, const CgState* st,
                           hipStream_t s) {
  launch_sweep(h, c, r, e, ez, st, s, true);
  if (!h.profiling) {
    launch_sweep(h, c, r, e, ez, st, s, false);
    return;
  }
  if (h.ev_used + 2 > (int)h.ev_pool.size()) {
    for (int t = 0; t < 64; ++t) {
      hipEvent_t ev;
      DDG_HIP(hipEventCreate(&ev));
      h.ev_pool.push_back(ev);
    }
  }
  int idx = h.ev_used;
  h.ev_used += 2;
  {
    KernelEvents ke(h, h.ev_pool[idx], h.ev_pool[idx + 1]);
    launch_sweep(h, c, r, e, ez, st, s, false);
  }
  h.pending.push_back({idx, ez ? h.S.n_colours + c : c, h.cur_tag});
}

// One persistent sweep direction; when profiling, its dispatch carries an event pair.
static void flow_profiled(Handle& h, int dir, const double* r, double* e, const CgState* st, hipStream_t s) {
  if (!h.profiling) {
    launch_sweep_flow(h, dir, r, e, st, s);
    return;
  }
  if (h.ev_used + 2 > (int)h.ev_pool.size()) {
    for (int t = 0; t < 64; ++t) {
      hipEvent_t ev;
      DDG_HIP(hipEventCreate(&ev));
      h.ev_pool.push_back(ev);
    }
  }
  int idx = h.ev_used;
  h.ev_used += 2;
  {
    KernelEvents ke(h, h.ev_pool[idx], h.ev_pool[idx + 1]);
    launch_sweep_flow(h, dir, r, e, st, s);
  }
  h.pending.push_back({idx, 2 * h.S.n_colours + dir, h.cur_tag});
}

void launch_precond(Handle& h, const double* r, double* e, int32_t stages, bool guarded, hipStream_t s,
                    const CgState* guard) {
  const CgState* st = guard ? guard : (guarded ? h.cstate.as<CgState>() : nullptr);
  const int C = h.S.n_colours;
  const int total = 2 * C + 1;
  if (stages < 0 || stages > total) stages = total;
  launch_fill(e, 0.0, h.S.n, s);
  if (h.flow_ok && stages == total) {
    // whole application: each sweep direction as one persistent launch
    flow_profiled(h, 0, r, e, st, s);
    launch_coarse(h, r, e, st, s);
    flow_profiled(h, 1, r, e, st, s);
    return;
  }
  int done = 0;
  for (int c = 0; c < C && done < stages; ++c, ++done) sweep_profiled(h, c, r, e, c == 0, st, s);
  if (done < stages) {
    launch_coarse(h, r, e, st, s);
    ++done;
  }
  for (int c = C - 1; c >= 0 && done < stages; --c, ++done) sweep_profiled(h, c, r, e, false, st, s);
}

}  // namespace ddg
