// Symmetric matrix-vector product from packed lower tiles, one wave per tile.
//
// A symmetric b x b matrix is stored as its lower-triangular T x T tiles
// (I >= J, row-major tile order I(I+1)/2 + J); diagonal tiles are stored in
// full (symmetrised), rows and columns beyond b are zero.  Inside a tile the
// 64 lanes form an 8 x 8 grid of S x S sub-tiles (S = T/8): lane L owns the
// sub-tile with rows lane_p(L)*S.. and columns lane_q(L)*S.., where q is made of
// lane bits {0,1,3} and p of lane bits {2,4,5}.  Inside its sub-tile the lane's
// register (i, j) holds row i ^ sq and column j ^ sp, with sq = q >> (3 - log2 S)
// and sp = p >> (3 - log2 S) (the coordinate bits the butterfly splits on): this
// lane-dependent order makes every lane keep the same register half at each
// butterfly step below, so the reduction needs no selects.  The lane's S*S
// values are stored as consecutive 16-byte chunks interleaved across lanes:
// chunk m of lane L sits at element (m*64 + L)*E (E values per chunk), so each
// load instruction of a wave reads one contiguous 1 KiB line.
//
// An off-diagonal tile contributes M x_J to rows I and M^T x_I to rows J, so
// each stored value is read once and used twice.  A diagonal tile may be stored
// compact: only the sub-tiles of the lanes with p >= q (36 of 64), the others
// being transposes of stored ones; kept lane L's chunk m then sits at element
// (m*36 + c(L))*E, c(L) = the number of kept lanes below L.  The tiles of a
// level's last tile-row likewise keep only the lanes whose sub-tile rows lie
// inside the level (see last_row_subtiles).  A compact diagonal tile's kept
// off-diagonal sub-tiles then contribute to the rows through both M x (row
// butterfly) and M^T x (column butterfly), like an off-diagonal tile.  Row partials are reduced
// across the 8 lanes that share p, column partials across the 8 lanes that
// share q, by butterfly halving.  With the bit assignment above the row
// butterfly only needs lane exchanges xor 8, 2, 1 (DPP moves inside a 16-lane
// row, no LDS traffic) and the column butterfly xor 32, 16, 4.
#pragma once

#include "device_util.hpp"

namespace ddg {

constexpr int kDiagLanes = 36;   // lanes that keep a sub-tile of a compact diagonal tile

template <class FT, int T>
struct TileGeom {
  static constexpr int S = T / 8;                                    // sub-tile edge
  static constexpr int SS = S * S;                                   // values per lane
  static constexpr int TD = kDiagLanes * SS;                         // values of a compact diagonal tile
  static constexpr int E = (16 / (int)sizeof(FT)) < SS ? (16 / (int)sizeof(FT)) : SS;  // values per chunk
  static constexpr int NCH = SS / E;                                 // chunks per lane
  static constexpr int LOGS = (S == 8) ? 3 : (S == 4 ? 2 : 1);
};

// Sub-tile coordinates of a lane.
__host__ __device__ constexpr int lane_q(int lane) { return (lane & 3) | ((lane >> 1) & 4); }
__host__ __device__ constexpr int lane_p(int lane) { return ((lane >> 2) & 1) | ((lane >> 3) & 6); }

// The local factors store their diagonal tiles compact for tile edges 32 and 64.
// (At edge 16, half of a typical level's tiles are diagonal and the solve is
// bound by latency, not bytes: the idle lanes cost more than the bytes saved.)
__host__ __device__ constexpr bool compact_diag(int T) { return T >= 32; }

// Short last tile-row.  The last tile-row of a b-row level holds h = b - (nt-1) T
// rows, i.e. data in its first ph = ceil(h / S) sub-tile rows; its tiles keep only
// the lanes with p < ph (the other lanes' sub-tiles are rows past b, all zero).
// Its off-diagonal tiles keep 8 ph lanes; its diagonal tile keeps the lanes with
// q <= p < ph when diagonal tiles are compact, else those with p, q < ph.  With
// ph = 8 these are the full and compact tiles of the other rows.
// Like compact diagonal tiles, short last rows are used at tile edges 32 and 64 only
// (at edge 16 a level has many small tiles and the per-tile work of finding the kept
// lanes costs more than the bytes save); at edge 16 ph is 8.
__host__ __device__ constexpr bool short_last_row(int T) { return T >= 32; }
__host__ __device__ inline int last_row_subtiles(int32_t b, int32_t T) {
  if (!short_last_row(T)) return 8;
  const int nt = (b + T - 1) / T, S = T / 8;
  return (b - (nt - 1) * T + S - 1) / S;
}

// Lanes kept by a tile with pmax sub-tile rows of data (diag: a diagonal tile,
// compact or full per cd).
__host__ __device__ constexpr unsigned long long kept_lanes(int pmax, bool diag, bool cd) {
  unsigned long long m = 0;
  for (int p = 0; p < pmax; ++p)
    for (int q = 0; q < 8; ++q) {
      if (diag && (cd ? q > p : q >= pmax)) continue;
      m |= 1ull << (((p & 1) << 2) | ((p >> 1) << 4) | (q & 3) | ((q >> 2) << 3));
    }
  return m;
}

// kept_lanes for a run-time pmax in 1..8 (each case folds to a constant).
template <bool CD>
__host__ __device__ inline unsigned long long kept_lanes_rt(int pmax, bool diag) {
  switch (pmax) {
    case 1: return diag ? kept_lanes(1, true, CD) : kept_lanes(1, false, CD);
    case 2: return diag ? kept_lanes(2, true, CD) : kept_lanes(2, false, CD);
    case 3: return diag ? kept_lanes(3, true, CD) : kept_lanes(3, false, CD);
    case 4: return diag ? kept_lanes(4, true, CD) : kept_lanes(4, false, CD);
    case 5: return diag ? kept_lanes(5, true, CD) : kept_lanes(5, false, CD);
    case 6: return diag ? kept_lanes(6, true, CD) : kept_lanes(6, false, CD);
    case 7: return diag ? kept_lanes(7, true, CD) : kept_lanes(7, false, CD);
    default: return diag ? kept_lanes(8, true, CD) : kept_lanes(8, false, CD);
  }
}

// Lanes kept by tile (I, J) of a level with nt tile-rows and ph data sub-tile rows
// in its last tile-row (all 64 for a full tile).
template <int T>
__host__ __device__ inline unsigned long long tile_lanes(int I, int J, int nt, int ph) {
  constexpr bool CD = compact_diag(T);
  if (I < nt - 1) return I == J ? kept_lanes(8, true, CD) : ~0ull;
  return kept_lanes_rt<CD>(ph, I == J);
}

// Elements of the packed lower tiles of a b-row level of the local factors.
__host__ __device__ inline int64_t level_elems(int32_t b, int32_t T) {
  const int64_t nt = (b + T - 1) / T, S = T / 8, ph = last_row_subtiles(b, T);
  const int64_t dl = compact_diag(T) ? kDiagLanes : 64;
  const int64_t last_diag = compact_diag(T) ? ph * (ph + 1) / 2 : ph * ph;
  const int64_t lanes = (nt - 1) * (nt - 2) / 2 * 64 + (nt - 1) * dl + (nt - 1) * 8 * ph + last_diag;
  return lanes * S * S;
}

// Element offset of tile t = (I, J) of a level of the local factors with nt
// tile-rows and ph data sub-tile rows in the last one (row-major lower order).
template <class FT, int T>
__host__ __device__ inline int64_t tile_off(int t, int I, int J, int nt, int ph) {
  using G = TileGeom<FT, T>;
  const int tr = I < nt - 1 ? t : (nt - 1) * nt / 2;  // first tile of the last row
  int64_t off = (int64_t)tr * T * T;
  if constexpr (compact_diag(T)) off -= (int64_t)(I < nt - 1 ? I : nt - 1) * (T * T - G::TD);
  if (I == nt - 1) off += (int64_t)J * 8 * ph * G::SS;
  return off;
}

// Element offset (within a tile) of sub-tile value (a, b) of lane L.
template <class FT, int T>
__host__ __device__ inline int tile_elem(int lane, int a, int b) {
  using G = TileGeom<FT, T>;
  int e = a * G::S + b;
  return ((e / G::E) * 64 + lane) * G::E + (e % G::E);
}

// Inverse of tile_elem: element offset within a tile -> (row, col) within the tile.
template <class FT, int T>
__host__ __device__ inline void tile_rc(int within, int& row, int& col) {
  using G = TileGeom<FT, T>;
  const int chunk = within / G::E;
  const int lane = chunk % 64;
  const int e = (chunk / 64) * G::E + within % G::E;
  const int p = lane_p(lane), q = lane_q(lane);
  row = p * G::S + ((e / G::S) ^ (q >> (3 - G::LOGS)));
  col = q * G::S + ((e % G::S) ^ (p >> (3 - G::LOGS)));
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

// Load the lane's values of a tile that stores nk lanes' sub-tiles, this lane's
// (if kept) as the c-th of them: chunk m at element (m * nk + c) * E; zeros when
// not kept.  A full tile is (kept, c, nk) = (true, lane, 64).
template <class FT, int T>
__device__ inline void load_subtile_at(const FT* __restrict__ tile, bool kept, int c, int nk,
                                       FT (&v)[TileGeom<FT, T>::SS]) {
  using G = TileGeom<FT, T>;
  constexpr int BYTES = G::E * (int)sizeof(FT);
  if (kept) {
#pragma unroll
    for (int m = 0; m < G::NCH; ++m) {
      const FT* src = tile + (m * nk + c) * G::E;
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
  } else {
#pragma unroll
    for (int u = 0; u < G::SS; ++u) v[u] = Store<FT>::from(0.0);
  }
}

// Value of the lane `lane ^ MASK` (MASK in {1, 2, 4, 8, 16, 32}).
template <int MASK>
__device__ inline int xor_lane_i32(int x) {
  if constexpr (MASK == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
  else if constexpr (MASK == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // quad_perm 2,3,0,1
  else if constexpr (MASK == 8) return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
  else if constexpr (MASK == 4) return __builtin_amdgcn_ds_swizzle(x, 0x1F | (4 << 10));
  else if constexpr (MASK == 16) return __builtin_amdgcn_ds_swizzle(x, 0x1F | (16 << 10));
  else return __shfl_xor(x, MASK, 64);
}

template <int MASK>
__device__ inline float xor_lane(float x) {
  return __int_as_float(xor_lane_i32<MASK>(__float_as_int(x)));
}

template <int MASK>
__device__ inline double xor_lane(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = xor_lane_i32<MASK>((int)(b & 0xffffffffLL));
  const int hi = xor_lane_i32<MASK>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One halving step of the butterfly: every lane keeps v[0..H) and adds the
// partner's v[H..2H), which holds the same rows because of the XOR storage
// order (see the layout note above).
template <int MASK, class AT, int H, int N>
__device__ inline void halve(AT (&v)[N]) {
#pragma unroll
  for (int i = 0; i < H; ++i) v[i] = v[i] + xor_lane<MASK>(v[i + H]);
}

// Reduce S values held by each of the 8 lanes of a group whose 3-bit
// coordinate c lives at the lane bits selected by masks (M2, M1, M0), most
// significant first.  Value i of the lane with coordinate c is logical entry
// i ^ (c >> (3 - LOGS)).  Afterwards the lane holds the group-total of logical
// entry c >> (3 - LOGS); `writer` is true for exactly one lane per entry.
template <class AT, int S, int LOGS, int M2, int M1, int M0>
__device__ inline AT group_reduce_scatter(AT (&v)[S], int c, bool& writer) {
  if constexpr (LOGS >= 1) halve<M2, AT, S / 2>(v);
  if constexpr (LOGS >= 2) halve<M1, AT, S / 4>(v);
  if constexpr (LOGS >= 3) halve<M0, AT, S / 8>(v);
  AT s = v[0];
  // remaining all-reduce steps when S < 8
  if constexpr (LOGS < 2) s += xor_lane<M1>(s);
  if constexpr (LOGS < 3) s += xor_lane<M0>(s);
  writer = (c & ((1 << (3 - LOGS)) - 1)) == 0;
  return s;
}

// Contributions of tile (I, J), whose values this lane holds in `m`:
//   rowslot[0..T) = (M x_J) over the tile's rows,
//   colslot[0..T) = (M^T x_I) over the tile's columns (off-diagonal tiles; with
//                   CD, also compact diagonal tiles, where it holds the
//                   contribution of the sub-tiles below the diagonal to the rows
//                   of their columns).
// x is indexed from the block's first row.  The slots are written, not
// accumulated, so the final sum over tiles has a fixed order.  The work is
// written as two phases: the lane's products, then the butterflies and stores.

// Phase 1: the lane's row and column partial sums of its sub-tile.
template <class FT, class AT, int T, bool CD = false>
__device__ inline void symv_tile_partials(const FT (&m)[TileGeom<FT, T>::SS], int I, int J,
                                          const AT* __restrict__ x, int lane, AT (&rowp)[TileGeom<FT, T>::S],
                                          AT (&colp)[TileGeom<FT, T>::S]) {
  using G = TileGeom<FT, T>;
  constexpr int S = G::S;
  const int p = lane_p(lane), q = lane_q(lane);
  const int pm = p >> (3 - G::LOGS), qm = q >> (3 - G::LOGS);
  // register (i, j) holds row p*S + (i ^ qm) and column q*S + (j ^ pm)
  AT xr[S], xc[S];
#pragma unroll
  for (int j = 0; j < S; ++j) xr[j] = x[J * T + q * S + (j ^ pm)];
#pragma unroll
  for (int i = 0; i < S; ++i) xc[i] = x[I * T + p * S + (i ^ qm)];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    rowp[i] = 0;
    colp[i] = 0;
  }
#pragma unroll
  for (int i = 0; i < S; ++i) {
#pragma unroll
    for (int j = 0; j < S; ++j) {
      AT mv = Store<FT>::to_acc(m[i * S + j]);
      rowp[i] += mv * xr[j];
      colp[j] += mv * xc[i];
    }
  }
  if constexpr (CD) {
    // a diagonal sub-tile already gave its rows through M x
    if (I == J && p == q) {
#pragma unroll
      for (int j = 0; j < S; ++j) colp[j] = 0;
    }
  }
}

// Phase 2: butterflies over the lanes that share rows (columns) and the slot stores.
template <class FT, class AT, int T, bool CD = false>
__device__ inline void symv_tile_store(int I, int J, AT (&rowp)[TileGeom<FT, T>::S],
                                       AT (&colp)[TileGeom<FT, T>::S], AT* __restrict__ rowslot,
                                       AT* __restrict__ colslot, int lane, bool valid) {
  using G = TileGeom<FT, T>;
  constexpr int S = G::S;
  const int p = lane_p(lane), q = lane_q(lane);
  bool w;
  AT rs = group_reduce_scatter<AT, S, G::LOGS, 8, 2, 1>(rowp, q, w);
  if (valid && w) rowslot[p * S + (q >> (3 - G::LOGS))] = rs;
  AT cs = group_reduce_scatter<AT, S, G::LOGS, 32, 16, 4>(colp, p, w);
  if (valid && (CD || I != J) && w) colslot[q * S + (p >> (3 - G::LOGS))] = cs;
}

template <class FT, class AT, int T, bool CD = false>
__device__ inline void symv_tile_slots(const FT (&m)[TileGeom<FT, T>::SS], int I, int J,
                                       const AT* __restrict__ x, AT* __restrict__ rowslot,
                                       AT* __restrict__ colslot, int lane, bool valid) {
  using G = TileGeom<FT, T>;
  AT rowp[G::S], colp[G::S];
  symv_tile_partials<FT, AT, T, CD>(m, I, J, x, lane, rowp, colp);
  symv_tile_store<FT, AT, T, CD>(I, J, rowp, colp, rowslot, colslot, lane, valid);
}

// Tile (I, J) of linear index t in row-major lower order.
__host__ __device__ inline void tile_ij(int t, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * t + 1.0f) - 1.0f) * 0.5f);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

// Fixed-order sum of the slots of output row r (0 <= r < nt*T) of a block with
// nt tile rows; slots of tile t sit at [2t][T] (rows) and [2t+1][T] (columns):
// sum_{J<=I} rowslot(I,J) (+ colslot(I,I) with compact diagonal tiles)
// + sum_{J>I} colslot(J,I), I = r/T.
template <class AT, int T, bool CD = false>
__device__ inline AT sum_slots(const AT* __restrict__ slots, int nt, int r) {
  const int I = r / T, rr = r % T;
  AT s = 0;
  for (int J = 0; J <= I; ++J) s += slots[(2 * (I * (I + 1) / 2 + J)) * T + rr];
  if constexpr (CD) s += slots[(2 * (I * (I + 1) / 2 + I) + 1) * T + rr];
  for (int J = I + 1; J < nt; ++J) s += slots[(2 * (J * (J + 1) / 2 + I) + 1) * T + rr];
  return s;
}

// As sum_slots, restricted to the tiles t0 <= t < t1 whose slots sit at
// [2(t - t0)][T] (rows) and [2(t - t0) + 1][T] (columns); same tile order.
template <class AT, int T, bool CD = false>
__device__ inline AT sum_slots_range(const AT* __restrict__ slots, int nt, int r, int t0, int t1) {
  const int I = r / T, rr = r % T;
  AT s = 0;
  const int a0 = I * (I + 1) / 2;
  for (int J = 0; J <= I; ++J) {
    const int t = a0 + J;
    if (t >= t0 && t < t1) s += slots[(2 * (t - t0)) * T + rr];
  }
  if constexpr (CD) {
    const int t = a0 + I;
    if (t >= t0 && t < t1) s += slots[(2 * (t - t0) + 1) * T + rr];
  }
  for (int J = I + 1; J < nt; ++J) {
    const int t = J * (J + 1) / 2 + I;
    if (t >= t0 && t < t1) s += slots[(2 * (t - t0) + 1) * T + rr];
  }
  return s;
}

}  // namespace ddg
