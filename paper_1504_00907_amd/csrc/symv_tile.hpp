// Symmetric matrix-vector product from packed lower tiles, one wave per tile.
//
// A symmetric b x b matrix is stored as its lower-triangular T x T tiles
// (I >= J, row-major tile order I(I+1)/2 + J); diagonal tiles are stored in
// full (symmetrised), rows and columns beyond b are zero.  Inside a tile the
// 64 lanes form an 8 x 8 grid: lane (p, q) = p*8 + q owns the S x S sub-tile
// (S = T/8) with rows p*S.. and columns q*S..  Its S*S values are stored as
// consecutive 16-byte chunks interleaved across lanes: chunk m of lane L sits
// at element (m*64 + L)*E (E values per chunk), so each load instruction of a
// wave reads one contiguous 1 KiB line.
//
// An off-diagonal tile contributes M x_J to rows I and M^T x_I to rows J, so
// each stored value is read once and used twice.  Row partials are reduced
// across the 8 lanes that share p (lane bits 0-2), column partials across the
// 8 lanes that share q (bits 3-5), by butterfly halving: 2*log2(S)+... shuffles
// per tile instead of a full 64-lane reduction per row.
#pragma once

#include "device_util.hpp"

namespace ddg {

template <class FT, int T>
struct TileGeom {
  static constexpr int S = T / 8;                                    // sub-tile edge
  static constexpr int SS = S * S;                                   // values per lane
  static constexpr int E = (16 / (int)sizeof(FT)) < SS ? (16 / (int)sizeof(FT)) : SS;  // values per chunk
  static constexpr int NCH = SS / E;                                 // chunks per lane
  static constexpr int LOGS = (S == 8) ? 3 : (S == 4 ? 2 : 1);
};

// Element offset (within a tile) of sub-tile value (a, b) of lane L.
template <class FT, int T>
__host__ __device__ inline int tile_elem(int lane, int a, int b) {
  using G = TileGeom<FT, T>;
  int e = a * G::S + b;
  return ((e / G::E) * 64 + lane) * G::E + (e % G::E);
}

// Load the lane's S*S values of one tile.
template <class FT, int T>
__device__ inline void load_subtile(const FT* __restrict__ tile, int lane, FT (&v)[TileGeom<FT, T>::SS]) {
  using G = TileGeom<FT, T>;
  constexpr int BYTES = G::E * (int)sizeof(FT);
#pragma unroll
  for (int m = 0; m < G::NCH; ++m) {
    const FT* src = tile + (m * 64 + lane) * G::E;
    if constexpr (BYTES == 16) {
      uint4 raw = *reinterpret_cast<const uint4*>(src);
      const FT* w = reinterpret_cast<const FT*>(&raw);
#pragma unroll
      for (int u = 0; u < G::E; ++u) v[m * G::E + u] = w[u];
    } else if constexpr (BYTES == 8) {
      uint2 raw = *reinterpret_cast<const uint2*>(src);
      const FT* w = reinterpret_cast<const FT*>(&raw);
#pragma unroll
      for (int u = 0; u < G::E; ++u) v[m * G::E + u] = w[u];
    } else {
#pragma unroll
      for (int u = 0; u < G::E; ++u) v[m * G::E + u] = src[u];
    }
  }
}

// Reduce S values held by each of the 8 lanes of a group whose coordinate c
// (0..7) sits at lane bits with unit stride `unit` (1 or 8).  Afterwards the
// lane holds the group-total of value index c >> (3 - LOGS); `writer` is true
// for exactly one lane per index.
template <class AT, int S, int LOGS>
__device__ inline AT group_reduce_scatter(AT (&v)[S], int c, int unit, bool& writer) {
  // halving steps with masks 4u, 2u, u (first LOGS of them)
  int len = S;
#pragma unroll
  for (int st = 0; st < LOGS; ++st) {
    const int mask = (4 >> st) * unit;
    const int hi = (c >> (2 - st)) & 1;
    const int half = len >> 1;
#pragma unroll
    for (int i = 0; i < S / 2; ++i) {
      if (i < half) {
        AT mine = hi ? v[i + half] : v[i];
        AT other = hi ? v[i] : v[i + half];
        v[i] = mine + __shfl_xor(other, mask, 64);
      }
    }
    len = half;
  }
  AT s = v[0];
  // remaining all-reduce steps
#pragma unroll
  for (int st = LOGS; st < 3; ++st) {
    const int mask = (4 >> st) * unit;
    s += __shfl_xor(s, mask, 64);
  }
  writer = (c & ((1 << (3 - LOGS)) - 1)) == 0;
  return s;
}

// One wave: contributions of tile (I, J) to out (a per-wave LDS row of partial sums).
// x is the input vector (LDS), indexed from the block's first row.
template <class FT, class AT, int T>
__device__ inline void symv_one_tile(const FT* __restrict__ tile, int I, int J, const AT* __restrict__ x,
                                     AT* __restrict__ out, int lane) {
  using G = TileGeom<FT, T>;
  constexpr int S = G::S;
  FT m[G::SS];
  load_subtile<FT, T>(tile, lane, m);
  const int p = lane >> 3, q = lane & 7;
  AT xr[S], xc[S];
#pragma unroll
  for (int b = 0; b < S; ++b) xr[b] = x[J * T + q * S + b];
#pragma unroll
  for (int a = 0; a < S; ++a) xc[a] = x[I * T + p * S + a];
  AT rowp[S], colp[S];
#pragma unroll
  for (int a = 0; a < S; ++a) {
    rowp[a] = 0;
    colp[a] = 0;
  }
#pragma unroll
  for (int a = 0; a < S; ++a) {
#pragma unroll
    for (int b = 0; b < S; ++b) {
      AT mv = Store<FT>::to_acc(m[a * S + b]);
      rowp[a] += mv * xr[b];
      colp[b] += mv * xc[a];
    }
  }
  bool w;
  AT rs = group_reduce_scatter<AT, S, G::LOGS>(rowp, q, 1, w);
  if (w) out[I * T + p * S + (q >> (3 - G::LOGS))] += rs;
  if (I != J) {
    AT cs = group_reduce_scatter<AT, S, G::LOGS>(colp, p, 8, w);
    if (w) out[J * T + q * S + (p >> (3 - G::LOGS))] += cs;
  }
}

// Tile (I, J) of linear index t in row-major lower order.
__device__ inline void tile_ij(int t, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

}  // namespace ddg
