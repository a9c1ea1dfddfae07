// Device helpers: fixed-order wave64/block reductions, storage-type conversions and
// CSR row dots by groups of lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <type_traits>

namespace ddg {

// Butterfly sum over the 64 lanes of a wave; every lane receives the same value
// and the summation order is fixed, so the result is reproducible.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a workgroup of NT threads (NT multiple of 64); result valid in thread 0.
template <int NT>
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  __syncthreads();
  return s;
}

// Sum of np partials by one workgroup in a fixed order; result valid in thread 0.
template <int NT>
__device__ inline double sum_partials(const double* __restrict__ part, int np, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += NT) acc += part[i];
  return block_sum<NT>(acc, red);
}

// Storage conversions for the local factors.
template <class T> struct Store;
template <> struct Store<double> {
  __device__ static double to_acc(double x) { return x; }
  __device__ static double from(double x) { return x; }
};
template <> struct Store<float> {
  __device__ static float to_acc(float x) { return x; }
  __device__ static float from(double x) { return (float)x; }
};
template <> struct Store<__hip_bfloat16> {
  __device__ static float to_acc(__hip_bfloat16 x) { return __bfloat162float(x); }
  __device__ static __hip_bfloat16 from(double x) { return __float2bfloat16((float)x); }
};

// Dot of CSR row g with x by a group of L consecutive lanes of a wave (L a power
// of two, at most 16): lane j of the group takes the entries j, j + L, ... in
// order, then an xor butterfly over the group adds the L partials, so every lane
// of the group returns the same reproducible value.  L = 1 is the plain
// sequential row sum.  All lanes of a group must be active together.
// Rows of at most kShortRow entries (stencils) issue all their loads at once,
// predicated, and then combine them in the stored order.
constexpr int kShortRow = 8;

// acc - sum_t v_t x_{c_t} over CSR row g, the entries subtracted in order.
__device__ inline double row_sub(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                 const double* __restrict__ v, const double* __restrict__ x, int64_t g,
                                 double acc) {
  const int64_t t0 = rp[g], t1 = rp[g + 1];
  if (t1 - t0 <= kShortRow) {
    int c[kShortRow];
    double a[kShortRow], xv[kShortRow];
#pragma unroll
    for (int q = 0; q < kShortRow; ++q) {
      c[q] = 0;
      a[q] = 0.0;
      if (t0 + q < t1) {
        c[q] = ci[t0 + q];
        a[q] = v[t0 + q];
      }
    }
#pragma unroll
    for (int q = 0; q < kShortRow; ++q) xv[q] = (t0 + q < t1) ? x[c[q]] : 0.0;
#pragma unroll
    for (int q = 0; q < kShortRow; ++q)
      if (t0 + q < t1) acc -= a[q] * xv[q];
    return acc;
  }
  for (int64_t t = t0; t < t1; ++t) acc -= v[t] * x[ci[t]];
  return acc;
}

template <int L>
__device__ inline double row_dot_l(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                   const double* __restrict__ v, const double* __restrict__ x, int64_t g,
                                   int j) {
  double s = 0.0;
  const int64_t t0 = rp[g], t1 = rp[g + 1];
  if (L == 1 && t1 - t0 <= kShortRow) {
    int c[kShortRow];
    double a[kShortRow], xv[kShortRow];
#pragma unroll
    for (int q = 0; q < kShortRow; ++q) {
      c[q] = 0;
      a[q] = 0.0;
      if (t0 + q < t1) {
        c[q] = ci[t0 + q];
        a[q] = v[t0 + q];
      }
    }
#pragma unroll
    for (int q = 0; q < kShortRow; ++q) xv[q] = (t0 + q < t1) ? x[c[q]] : 0.0;
#pragma unroll
    for (int q = 0; q < kShortRow; ++q)
      if (t0 + q < t1) s += a[q] * xv[q];
    return s;
  }
#pragma unroll 4
  for (int64_t t = t0 + j; t < t1; t += L) s += v[t] * x[ci[t]];
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// row_dot_l<L> for a run-time group width L > 1 (a power of two, at most 16): the
// same products, added in the same order, so both return the same bits.
__device__ inline double row_dot_rt(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                    const double* __restrict__ v, const double* __restrict__ x, int64_t g,
                                    int j, int L) {
  double s = 0.0;
  const int64_t t0 = rp[g], t1 = rp[g + 1];
  for (int64_t t = t0 + j; t < t1; t += L) s += v[t] * x[ci[t]];
  for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// ---------------------------------------------------------------------------
// Diagonal (DIA) storage of a stencil operator, used for every row dot when each
// system's stored entries lie on at most kDiaMax offset pairs +-o (5-, 7- and
// 13-point stencils).  The values are symmetric bit for bit (checked when they
// are filled), so only the diagonal and the upper diagonals are stored:
// A[g, g] = diag[g], A[g, g + o_d] = A[g + o_d, g] = up[d n + g], zero where the
// CSR row has no such entry.  A row is read back in its sorted-column order
// (lower diagonals by descending offset, the diagonal, upper ones by ascending
// offset), so every sum equals the CSR one bit for bit (a missing entry adds
// 0 * x).  Each system of a batch has its own offsets and row range.
constexpr int kDiaMax = 6;

struct DiaSys {
  int64_t lo, hi;        // rows of the system
  int32_t nd;            // upper diagonals (<= kDiaMax)
  int32_t off[kDiaMax];  // ascending positive offsets
  int32_t pad;
};

struct DiaView {
  const double* diag;    // n; null when the handle uses CSR rows
  const double* up;      // kDiaMax x n (diagonal d at up + d n)
  const DiaSys* sys;     // per system
  int64_t n;
  int32_t nb;
};

// System holding row g (binary search over the row ranges).
__device__ inline int dia_system_of(const DiaView& D, int64_t g) {
  int lo = 0, hi = D.nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (D.sys[mid].lo <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Loads the entries of row g in sorted-column order into a[], x values into xv[]:
// slots 0..nd-1 the lower diagonals (largest offset first), slot kDiaMax the
// diagonal, slots kDiaMax+1.. the upper ones; a slot whose neighbour lies
// outside the system holds 0.
__device__ inline void dia_row_load(const DiaView& D, const DiaSys& s, const double* __restrict__ x, int64_t g,
                                    double (&a)[2 * kDiaMax + 1], double (&xv)[2 * kDiaMax + 1]) {
  const int nd = s.nd;
#pragma unroll
  for (int q = 0; q < kDiaMax; ++q) {
    a[q] = 0.0;
    xv[q] = 0.0;
    const int d = nd - 1 - q;
    if (d >= 0) {
      const int64_t c = g - s.off[d];
      if (c >= s.lo) {
        a[q] = D.up[(int64_t)d * D.n + c];
        xv[q] = x[c];
      }
    }
  }
  a[kDiaMax] = D.diag[g];
  xv[kDiaMax] = x[g];
#pragma unroll
  for (int q = 0; q < kDiaMax; ++q) {
    a[kDiaMax + 1 + q] = 0.0;
    xv[kDiaMax + 1 + q] = 0.0;
    if (q < nd) {
      const int64_t c = g + s.off[q];
      if (c < s.hi) {
        a[kDiaMax + 1 + q] = D.up[(int64_t)q * D.n + g];
        xv[kDiaMax + 1 + q] = x[c];
      }
    }
  }
}

// acc - (A x)_g, the entries subtracted in sorted-column order (as row_sub).
__device__ inline double dia_row_sub(const DiaView& D, const DiaSys& s, const double* __restrict__ x, int64_t g,
                                     double acc) {
  double a[2 * kDiaMax + 1], xv[2 * kDiaMax + 1];
  dia_row_load(D, s, x, g, a, xv);
#pragma unroll
  for (int q = 0; q < 2 * kDiaMax + 1; ++q)
    if (q < kDiaMax ? q < s.nd : q == kDiaMax || q - kDiaMax - 1 < s.nd) acc -= a[q] * xv[q];
  return acc;
}

// (A x)_g, the products added in sorted-column order (as row_dot_l<1>).
__device__ inline double dia_row_dot(const DiaView& D, const DiaSys& s, const double* __restrict__ x, int64_t g) {
  double a[2 * kDiaMax + 1], xv[2 * kDiaMax + 1];
  dia_row_load(D, s, x, g, a, xv);
  double r = 0.0;
#pragma unroll
  for (int q = 0; q < 2 * kDiaMax + 1; ++q)
    if (q < kDiaMax ? q < s.nd : q == kDiaMax || q - kDiaMax - 1 < s.nd) r += a[q] * xv[q];
  return r;
}

// Calls f(std::integral_constant<int, L>{}) for the run-time lanes-per-row value.
template <class Fn>
inline void with_lanes(int L, Fn&& f) {
  switch (L) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 1>{}); break;
  }
}

}  // namespace ddg
