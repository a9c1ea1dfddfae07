// Coarse correction of the two-level preconditioner (Section 4 coarse problem,
// Section 6 multiplicative combination):
//     e += R0^T A0^{-1} R0 (r - A e)
// R0^T = blockdiag(Q_i) with Q_i the orthonormal basis of subdomain i, so
//   b0[off_i + m] = sum_{g in Omega_i} Q[g, m] (r - A e)_g        (restrict)
//   y = A0^{-1} b0                                                  (tiled symmetric GEMV)
//   e_g += sum_m Q[g, m] y[off_{part g} + m]                        (prolong)
// A0^{-1} is the explicit float64 inverse computed at setup; it is stored as
// lower 64 x 64 tiles and applied with one wave per tile, writing fixed
// per-tile partials that a second kernel sums in a fixed order.  With several
// independent systems A0 is block diagonal: system b owns the padded coarse
// rows [cblk_off[b], cblk_off[b+1]) and the tiles [tile_base[b], tile_base[b+1])
// of its own inverse; kernels skip the work of systems that have stopped.
#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

namespace {

constexpr int kRThreads = 256;

// Partial restriction over one chunk of the own rows of subdomain i (workgroup
// (c, i) takes rows [own_ptr[i] + c rch, ... + rch)), L lanes per CSR row:
//   rpart[i, c, m] = sum_{g in chunk} Q[g, m] (r - A e)_g,   m < kcnt[i]
// (waves in order after a butterfly per wave); empty chunks write zeros.
// KM: capacity of the per-thread column arrays and stride of rpart (kslots(k)).
template <int L, int KM>
__global__ void __launch_bounds__(kRThreads) k_coarse_restrict(
    const CgState* st, const int32_t* __restrict__ sub_inst, const int64_t* __restrict__ own_ptr,
    const int32_t* __restrict__ own_idx, const int32_t* __restrict__ kcnt, const double* __restrict__ Q, int kq,
    const int64_t* __restrict__ rp, const int32_t* __restrict__ ci, const double* __restrict__ val,
    DiaView D, const double* __restrict__ r, const double* __restrict__ e, int rch, double* __restrict__ rpart) {
  const int i = blockIdx.y, c = blockIdx.x;
  if (st && st[sub_inst[i]].done) return;
  __shared__ double red[kRThreads / 64][KM];
  const int ki = kcnt[i];
  double acc[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) acc[m] = 0.0;
  const int64_t t0 = own_ptr[i] + (int64_t)c * rch;
  const int64_t t1 = min(own_ptr[i + 1], t0 + rch);
  const int jl = threadIdx.x & (L - 1);
  if constexpr (L == 1) {
    // a thread's rows t, t + 256, ... four at a time: each stage's loads (row index,
    // row pointers, entries, e) go out for all four rows together; the rows are
    // still added in the same order
    constexpr int U = 4;
    for (int64_t t = t0 + threadIdx.x; t < t1; t += (int64_t)U * kRThreads) {
      int g[U];
      double sv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) g[u] = t + u * kRThreads < t1 ? own_idx[t + u * kRThreads] : -1;
      if (D.diag) {
        const DiaSys& sy = D.sys[sub_inst[i]];
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = g[u] >= 0 ? dia_row_sub(D, sy, e, g[u], r[g[u]]) : 0.0;
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) sv[u] = g[u] >= 0 ? row_sub(rp, ci, val, e, g[u], r[g[u]]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (g[u] < 0) continue;
        const double* qg = Q + (int64_t)g[u] * kq;
#pragma unroll
        for (int m = 0; m < KM; ++m)
          if (m < ki) acc[m] += qg[m] * sv[u];
      }
    }
  } else {
    for (int64_t t = t0 + threadIdx.x / L; t < t1; t += kRThreads / L) {
      const int g = own_idx[t];
      const double s = r[g] - row_dot_l<L>(rp, ci, val, e, g, jl);
      if (jl == 0) {
        const double* qg = Q + (int64_t)g * kq;
#pragma unroll
        for (int m = 0; m < KM; ++m)
          if (m < ki) acc[m] += qg[m] * s;
      }
    }
  }
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m < ki) {
      double v = wave_sum(acc[m]);
      if ((threadIdx.x & 63) == 0) red[wv][m] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < ki) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRThreads / 64; ++w) s += red[w][threadIdx.x];
    rpart[((int64_t)i * gridDim.x + c) * KM + threadIdx.x] = s;
  }
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
  if (m >= kcnt[i]) return;
  const double* p = rpart + (int64_t)i * nch * KM + m;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += p[(int64_t)c * KM];
  b0[koff[i] + m] = s;
}

// one wave per 64x64 float64 tile: row and column partials into per-tile slots
__global__ void __launch_bounds__(256) k_coarse_symv(const CgState* st, const int32_t* __restrict__ tile_inst,
                                                     const int64_t* __restrict__ tile_base,
                                                     const int64_t* __restrict__ cblk_off,
                                                     const double* __restrict__ tiles, int64_t ntiles,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ rowpart,
                                                     double* __restrict__ colpart) {
  constexpr int T = 64;
  using G = TileGeom<double, T>;
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const int b = tile_inst[t];
  if (st && st[b].done) return;
  int I, J;
  tile_ij((int)(t - tile_base[b]), I, J);
  double m[G::SS];
  load_subtile<double, T>(tiles + t * T * T, lane, m);
  symv_tile_slots<double, double, T>(m, I, J, x + cblk_off[b], rowpart + t * T, colpart + t * T, lane, true);
}

// y over the padded coarse rows; trow_inst gives the system of each 64-row tile row
__global__ void k_coarse_sum(const CgState* st, const int32_t* __restrict__ trow_inst,
                             const int64_t* __restrict__ tile_base, const int64_t* __restrict__ cblk_off,
                             const double* __restrict__ rowpart, const double* __restrict__ colpart,
                             int64_t nc_pad, double* __restrict__ y) {
  constexpr int T = 64;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nc_pad) return;
  const int b = trow_inst[row / T];
  if (st && st[b].done) return;
  const int64_t lr = row - cblk_off[b];
  const int I = (int)(lr / T), rr = (int)(lr % T);
  const int ntr = (int)((cblk_off[b + 1] - cblk_off[b]) / T);
  const double* rp = rowpart + tile_base[b] * T;
  const double* cp = colpart + tile_base[b] * T;
  double s = 0.0;
  for (int J = 0; J <= I; ++J) s += rp[((int64_t)I * (I + 1) / 2 + J) * T + rr];
  for (int J = I + 1; J < ntr; ++J) s += cp[((int64_t)J * (J + 1) / 2 + I) * T + rr];
  y[row] = s;
}

template <int KM>
__global__ void __launch_bounds__(256) k_coarse_prolong(const CgState* st, const int32_t* __restrict__ sub_inst,
                                 const int32_t* __restrict__ part,
                                 const int32_t* __restrict__ kcnt, const int64_t* __restrict__ koff,
                                 const double* __restrict__ Q, int kq, const double* __restrict__ y,
                                 double* __restrict__ e, int64_t n) {
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  // the row of Q (stride kq) is requested before the subdomain's count and offset
  // are known, so its loads do not wait behind that chain of lookups
  const double* qg = Q + g * kq;
  double q[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) q[m] = m < kq ? qg[m] : 0.0;
  const int i = part[g];
  if (st && st[sub_inst[i]].done) return;
  const int ki = kcnt[i];
  const double* yi = y + koff[i];
  double s = 0.0;
#pragma unroll
  for (int m = 0; m < KM; ++m)
    if (m < ki) s += q[m] * yi[m];
  e[g] += s;
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

}  // namespace

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
                       h.Q.as<double>(), h.k, h.rowptr.as<int64_t>(), h.col.as<int32_t>(), h.val.as<double>(),
                       dia_view(h), r, e, h.rch, h.ws.rpart);
  });
  hipLaunchKernelGGL(k_coarse_restrict_sum, dim3((unsigned)(((int64_t)S.n_parts * KM + 255) / 256)), dim3(256), 0,
                     s, st, sub_inst, h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(), h.ws.rpart, h.nch,
                     S.n_parts, KM, b0);
  if (h.inner) {
    // three levels: y = M0^{-1} b0, one application of the coarse level's two-level
    // preconditioner (its kernels skip work once this handle's system has stopped)
    launch_precond(*h.inner, b0, y, -1, false, s, st);
  } else {
  double* rowpart = h.ws.cpart;
  double* colpart = rowpart + h.ntiles * 64;
  hipLaunchKernelGGL(k_coarse_symv, dim3((unsigned)((h.ntiles + 3) / 4)), dim3(256), 0, s, st,
                     h.tile_inst.as<int32_t>(), h.tile_base_d.as<int64_t>(), h.cblk_off_d.as<int64_t>(),
                     h.A0inv_t.as<double>(), h.ntiles, b0, rowpart, colpart);
  hipLaunchKernelGGL(k_coarse_sum, dim3((unsigned)((h.nc_pad + 255) / 256)), dim3(256), 0, s, st,
                     h.trow_inst.as<int32_t>(), h.tile_base_d.as<int64_t>(), h.cblk_off_d.as<int64_t>(),
                     rowpart, colpart, h.nc_pad, y);
  }
  hipLaunchKernelGGL(k_coarse_prolong<KM>, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, s, st, sub_inst,
                     h.part.as<int32_t>(), h.kcnt_d.as<int32_t>(), h.koff_d.as<int64_t>(),
                     h.Q.as<double>(), h.k, y, e, S.n);
  DDG_HIP(hipGetLastError());
}

void launch_coarse(Handle& h, const double* r, double* e, const CgState* st, hipStream_t s) {
  if (h.nc == 0) return;
  DDG_REQUIRE(h.k <= kMaxGen, DDG_ERR_UNSUPPORTED, "at most 80 generating vectors");
  if (h.k <= 32) launch_coarse_k<32>(h, r, e, st, s);
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
