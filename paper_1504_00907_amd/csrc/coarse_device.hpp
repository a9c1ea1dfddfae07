// Device bodies of the coarse correction (Section 4 coarse problem, Section 6
// multiplicative combination), e += R0^T A0^{-1} R0 (r - A e): used by the
// one-launch-per-step kernels (kernels_coarse.hip) and by the persistent batched
// solve, with the same arithmetic in the same order.
#pragma once

#include "common.hpp"
#include "device_util.hpp"
#include "symv_tile.hpp"

namespace ddg {

constexpr int kRThreads = 256;

// The basis as the solve reads it: row t of the own-row order (the rows of
// subdomain 0, then of subdomain 1, ...; own_idx maps t to the global row),
// column m < kq, in 64-row tiles stored column-major, so that the 64 lanes of a
// wave reading one column of 64 consecutive own rows read 512 contiguous bytes.
__host__ __device__ inline int64_t q_own_at(int64_t t, int m, int kq) {
  return ((t >> 6) * kq + m) * 64 + (t & 63);
}

// Partial restriction over one chunk of the own rows of subdomain i (workgroup
// (c, i) takes rows [own_ptr[i] + c rch, ... + rch)), L lanes per CSR row:
//   rpart[i, c, m] = sum_{g in chunk} Q[g, m] (r - A e)_g,   m < kcnt[i]
// with the basis read from the own-row layout Qo (q_own_at)
// (waves in order after a butterfly per wave); empty chunks write zeros.
// KM: capacity of the per-thread column arrays and stride of rpart (kslots(k)).
// (the first kRThreads threads of the workgroup do the work; any others join the barrier)
template <int L, int KM>
__device__ inline void d_coarse_restrict(int i, int c, int nch, const int32_t* __restrict__ sub_inst,
                                         const int64_t* __restrict__ own_ptr, const int32_t* __restrict__ own_idx,
                                         const int32_t* __restrict__ kcnt, const double* __restrict__ Qo, int kq,
                                         const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                         const double* __restrict__ val, const DiaView D,
                                         const double* __restrict__ r, const double* __restrict__ e, int rch,
                                         double* __restrict__ rpart) {
  __shared__ double red[kRThreads / 64][KM];
  const int ki = kcnt[i];
  double acc[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) acc[m] = 0.0;
  const int64_t t0 = own_ptr[i] + (int64_t)c * rch;
  const int64_t t1 = threadIdx.x < kRThreads ? min(own_ptr[i + 1], t0 + rch) : t0;
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
        const double* qt = Qo + q_own_at(t + u * kRThreads, 0, kq);
#pragma unroll
        for (int m = 0; m < KM; ++m)
          if (m < ki) acc[m] += qt[m * 64] * sv[u];
      }
    }
  } else {
    for (int64_t t = t0 + threadIdx.x / L; t < t1; t += kRThreads / L) {
      const int g = own_idx[t];
      const double s = r[g] - row_dot_l<L>(rp, ci, val, e, g, jl);
      if (jl == 0) {
        const double* qt = Qo + q_own_at(t, 0, kq);
#pragma unroll
        for (int m = 0; m < KM; ++m)
          if (m < ki) acc[m] += qt[m * 64] * s;
      }
    }
  }
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < KM; ++m) {
    if (m < ki) {
      double v = wave_sum(acc[m]);
      if ((threadIdx.x & 63) == 0 && wv < kRThreads / 64) red[wv][m] = v;
    }
  }
  __syncthreads();
  if (threadIdx.x < ki) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRThreads / 64; ++w) s += red[w][threadIdx.x];
    rpart[((int64_t)i * nch + c) * KM + threadIdx.x] = s;
  }
}

// b0[koff[i] + m] = sum over the nch chunks of subdomain i, in chunk order (m < kcnt[i])
__device__ inline void d_coarse_restrict_sum_entry(int i, int m, const int32_t* __restrict__ kcnt,
                                                   const int64_t* __restrict__ koff, const double* __restrict__ rpart,
                                                   int nch, int KM, double* __restrict__ b0) {
  if (m >= kcnt[i]) return;
  const double* p = rpart + (int64_t)i * nch * KM + m;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += p[(int64_t)c * KM];
  b0[koff[i] + m] = s;
}

// one wave: tile t (of system b) of the packed inverse, row and column partials into its slots
__device__ inline void d_coarse_symv_tile(int64_t t, int b, const int64_t* __restrict__ tile_base,
                                          const int64_t* __restrict__ cblk_off, const double* __restrict__ tiles,
                                          const double* __restrict__ x, double* __restrict__ rowpart,
                                          double* __restrict__ colpart) {
  constexpr int T = 64;
  using G = TileGeom<double, T>;
  const int lane = threadIdx.x & 63;
  int I, J;
  tile_ij((int)(t - tile_base[b]), I, J);
  double m[G::SS];
  load_subtile<double, T>(tiles + t * T * T, lane, m);
  symv_tile_slots<double, double, T>(m, I, J, x + cblk_off[b], rowpart + t * T, colpart + t * T, lane, true);
}

// y[row] from the tile slots of system b, in a fixed order
__device__ inline void d_coarse_sum_row(int64_t row, int b, const int64_t* __restrict__ tile_base,
                                        const int64_t* __restrict__ cblk_off, const double* __restrict__ rowpart,
                                        const double* __restrict__ colpart, double* __restrict__ y) {
  constexpr int T = 64;
  const int64_t lr = row - cblk_off[b];
  const int I = (int)(lr / T), rr = (int)(lr % T);
  const int ntr = (int)((cblk_off[b + 1] - cblk_off[b]) / T);
  const double* rp = rowpart + tile_base[b] * T;
  const double* cp = colpart + tile_base[b] * T;
  // (the loads of eight terms go out together; the terms are added in order)
  constexpr int U = 8;
  double s = 0.0;
  const double* r0 = rp + (int64_t)I * (I + 1) / 2 * T + rr;   // tile (I, J) at r0 + J T
  int J = 0;
  for (; J + U <= I + 1; J += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = r0[(int64_t)(J + u) * T];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; J <= I; ++J) s += r0[(int64_t)J * T];
  J = I + 1;
  for (; J + U <= ntr; J += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = cp[((int64_t)(J + u) * (J + u + 1) / 2 + I) * T + rr];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; J < ntr; ++J) s += cp[((int64_t)J * (J + 1) / 2 + I) * T + rr];
  y[row] = s;
}

// e[g] += sum_m Q[g, m] y[koff[part g] + m] for the row g at position t of the
// own-row order (g = own_idx[t])
template <int KM>
__device__ inline void d_coarse_prolong_row(int64_t g, int64_t t, const CgState* st,
                                            const int32_t* __restrict__ sub_inst, const int32_t* __restrict__ part,
                                            const int32_t* __restrict__ kcnt, const int64_t* __restrict__ koff,
                                            const double* __restrict__ Qo, int kq, const double* __restrict__ y,
                                            double* __restrict__ e) {
  // the row of the basis is requested before the subdomain's count and offset are
  // known, so its loads do not wait behind that chain of lookups
  const double* qt = Qo + q_own_at(t, 0, kq);
  double q[KM];
#pragma unroll
  for (int m = 0; m < KM; ++m) q[m] = m < kq ? qt[m * 64] : 0.0;
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

}  // namespace ddg
