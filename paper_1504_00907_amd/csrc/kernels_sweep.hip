// Colour phase of the multiplicative Schwarz sweep (Section 6 update equation):
// for every subdomain i of one colour, concurrently,
//     e[set_i] += A_i^{-1} (r - A e)[set_i].
// Same-colour subdomains never touch each other's set or its neighbourhood
// (conflict colouring), so the phase is race-free and deterministic.
//
// Local solve: A_i is block tridiagonal over the levels of its ascending
// ordering.  The factorisation stores X_k = S_k^{-1} for the Schur complements
// S_0 = D_0, S_k = D_k - L_k X_{k-1} L_k^T (block LDL^T), so
//   forward:  t_k = X_k (b_k - L_k t_{k-1})
//   backward: x_K = t_K,  x_k = t_k - X_k (U_k x_{k+1})
// where L_k / U_k are the sparse couplings of block k to its lower / upper
// neighbour taken from A.  Each X_k product is a tiled symmetric GEMV
// (symv_tile.hpp) that streams the factor from HBM once per substitution.
#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

struct SweepArgs {
  const int32_t* subs;
  const int64_t* set_ptr;
  const int32_t* set_idx;
  const int32_t* sub_blk_ptr;
  const int32_t* blk_start;
  const int32_t* blk_size;
  const int64_t* blk_foff;
  const int64_t* lo_ptr;
  const int32_t* lo_col;
  const double* lo_val;
  const int64_t* up_ptr;
  const int32_t* up_col;
  const double* up_val;
  const int64_t* rp;
  const int32_t* ci;
  const double* val;
  const void* fac;
  const double* r;
  double* e;
  const CgState* st;
  int32_t e_zero;
  int32_t ldp;  // per-wave partial row length (>= max padded block rows)
};

template <class FT, class AT, int T, int NW>
__global__ void __launch_bounds__(NW * 64) k_sweep(SweepArgs a) {
  if (a.st && a.st->done) return;
  constexpr int NT = NW * 64;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int sub = a.subs[blockIdx.x];
  const int64_t s0 = a.set_ptr[sub];
  const int ni = (int)(a.set_ptr[sub + 1] - s0);
  AT* w = reinterpret_cast<AT*>(smem_raw);
  // layout: w[ni_pad] | tv[ldp] | part[NW][ldp]
  const int ni_pad = (ni + 3) & ~3;
  AT* tv = w + ni_pad;
  AT* part = tv + a.ldp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const FT* fac = static_cast<const FT*>(a.fac);

  // 1. gather the local residual b = (r - A e)[set]
  for (int j = tid; j < ni; j += NT) {
    const int g = a.set_idx[s0 + j];
    double acc = a.r[g];
    if (!a.e_zero) {
      for (int64_t t = a.rp[g]; t < a.rp[g + 1]; ++t) acc -= a.val[t] * a.e[a.ci[t]];
    }
    w[j] = (AT)acc;
  }
  __syncthreads();

  const int kb0 = a.sub_blk_ptr[sub];
  const int K = a.sub_blk_ptr[sub + 1] - kb0;

  auto block_symv = [&](int k) {
    const int b = a.blk_size[kb0 + k];
    const int nt = (b + T - 1) / T;
    const int ntiles = nt * (nt + 1) / 2;
    AT* mine = part + wave * a.ldp;
    for (int r = lane; r < nt * T; r += 64) mine[r] = 0;
    const FT* tiles = fac + a.blk_foff[kb0 + k];
    for (int t = wave; t < ntiles; t += NW) {
      int I, J;
      tile_ij(t, I, J);
      symv_one_tile<FT, AT, T>(tiles + (int64_t)t * T * T, I, J, tv, mine, lane);
    }
  };

  // 2. forward elimination
  for (int k = 0; k < K; ++k) {
    const int bs = a.blk_start[kb0 + k];
    const int b = a.blk_size[kb0 + k];
    const int nt = (b + T - 1) / T;
    for (int jj = tid; jj < nt * T; jj += NT) {
      AT y = 0;
      if (jj < b) {
        const int64_t row = s0 + bs + jj;
        y = w[bs + jj];
        for (int64_t t = a.lo_ptr[row]; t < a.lo_ptr[row + 1]; ++t)
          y -= (AT)a.lo_val[t] * w[a.lo_col[t]];
      }
      tv[jj] = y;
    }
    __syncthreads();
    block_symv(k);
    __syncthreads();
    for (int jj = tid; jj < b; jj += NT) {
      AT s = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) s += part[q * a.ldp + jj];
      w[bs + jj] = s;
    }
    __syncthreads();
  }

  // 3. backward substitution
  for (int k = K - 2; k >= 0; --k) {
    const int bs = a.blk_start[kb0 + k];
    const int b = a.blk_size[kb0 + k];
    const int nt = (b + T - 1) / T;
    for (int jj = tid; jj < nt * T; jj += NT) {
      AT v = 0;
      if (jj < b) {
        const int64_t row = s0 + bs + jj;
        for (int64_t t = a.up_ptr[row]; t < a.up_ptr[row + 1]; ++t)
          v += (AT)a.up_val[t] * w[a.up_col[t]];
      }
      tv[jj] = v;
    }
    __syncthreads();
    block_symv(k);
    __syncthreads();
    for (int jj = tid; jj < b; jj += NT) {
      AT s = 0;
#pragma unroll
      for (int q = 0; q < NW; ++q) s += part[q * a.ldp + jj];
      w[bs + jj] -= s;
    }
    __syncthreads();
  }

  // 4. scatter-add the correction
  for (int j = tid; j < ni; j += NT) {
    const int g = a.set_idx[s0 + j];
    a.e[g] += (double)w[j];
  }
}

namespace {

constexpr int kSweepWaves = 8;

template <class FT, class AT, int T>
void launch_sweep_t(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                    const CgState* st, hipStream_t s) {
  const Symbolic& S = h.S;
  int nsub = S.colour_ptr[colour + 1] - S.colour_ptr[colour];
  if (nsub == 0) return;
  SweepArgs a;
  a.subs = h.colour_subs.as<int32_t>() + S.colour_ptr[colour];
  a.set_ptr = h.set_ptr.as<int64_t>();
  a.set_idx = h.set_idx.as<int32_t>();
  a.sub_blk_ptr = h.sub_blk_ptr.as<int32_t>();
  a.blk_start = h.blk_start.as<int32_t>();
  a.blk_size = h.blk_size.as<int32_t>();
  a.blk_foff = h.blk_foff.as<int64_t>();
  a.lo_ptr = h.lo_ptr.as<int64_t>();
  a.lo_col = h.lo_col.as<int32_t>();
  a.lo_val = h.lo_val.as<double>();
  a.up_ptr = h.up_ptr.as<int64_t>();
  a.up_col = h.up_col.as<int32_t>();
  a.up_val = h.up_val.as<double>();
  a.rp = h.rowptr.as<int64_t>();
  a.ci = h.col.as<int32_t>();
  a.val = h.val.as<double>();
  a.fac = h.fac.p;
  a.r = r;
  a.e = e;
  a.st = st;
  a.e_zero = e_zero ? 1 : 0;
  const int maxpad = ((S.max_blk + T - 1) / T) * T;
  a.ldp = maxpad;
  const int ni_pad = (S.max_set + 3) & ~3;
  size_t lds = sizeof(AT) * ((size_t)ni_pad + (size_t)maxpad * (1 + kSweepWaves));
  auto kern = k_sweep<FT, AT, T, kSweepWaves>;
  DDG_REQUIRE((int64_t)lds <= h.dev_lds_limit, DDG_ERR_UNSUPPORTED,
              "local problem too large for on-chip storage (" + std::to_string(lds) + " bytes)");
  if (lds > 65536) DDG_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(kern, dim3(nsub), dim3(kSweepWaves * 64), lds, s, a);
  DDG_HIP(hipGetLastError());
}

template <class FT, class AT>
void launch_sweep_p(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                    const CgState* st, hipStream_t s) {
  switch (h.S.tile) {
    case 16: launch_sweep_t<FT, AT, 16>(h, colour, r, e, e_zero, st, s); break;
    case 32: launch_sweep_t<FT, AT, 32>(h, colour, r, e, e_zero, st, s); break;
    default: launch_sweep_t<FT, AT, 64>(h, colour, r, e, e_zero, st, s); break;
  }
}

}  // namespace

void launch_sweep(const Handle& h, int colour, const double* r, double* e, bool e_zero,
                  const CgState* st, hipStream_t s) {
  switch (h.opt.precision) {
    case DDG_MIXED_FP32: launch_sweep_p<float, float>(h, colour, r, e, e_zero, st, s); break;
    case DDG_MIXED_BF16: launch_sweep_p<__hip_bfloat16, float>(h, colour, r, e, e_zero, st, s); break;
    default: launch_sweep_p<double, double>(h, colour, r, e, e_zero, st, s); break;
  }
}

}  // namespace ddg
