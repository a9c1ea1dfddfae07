// C ABI of libddg: argument checks, device memory plan, setup orchestration
// and the PCG driver loop.  Every numeric step runs in the HIP kernels of the
// other translation units; this file only moves integers and pointers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <memory>

#include "common.hpp"
#include "symv_tile.hpp"

namespace ddg {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

void launch_coarse(Handle& h, const double* r, double* e, const CgState* st, hipStream_t s);

Handle::~Handle() {
  delete inner;
  for (auto ev : ev_pool) (void)hipEventDestroy(ev);
  if (h_state) (void)hipHostFree(h_state);
  if (h_cerr) (void)hipHostFree(h_cerr);
  if (side) (void)hipStreamDestroy(side);
}

namespace {

int64_t tile_bytes(int32_t b, int32_t T, int es) { return level_elems(b, T) * es; }

int storage_size(int precision) {
  return precision == DDG_MIXED_FP32 ? 4 : (precision == DDG_MIXED_BF16 ? 2 : 8);
}

void check_values(int64_t n, const int64_t* rp, const int32_t* ci, const double* val) {
  double amax = 0.0;
  for (int64_t t = 0; t < rp[n]; ++t) {
    DDG_REQUIRE(std::isfinite(val[t]), DDG_ERR_INVALID_ARG, "non-finite matrix value");
    amax = std::max(amax, std::fabs(val[t]));
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t t = rp[i]; t < rp[i + 1]; ++t) {
      const int32_t c = ci[t];
      if (c == i) {
        DDG_REQUIRE(val[t] > 0.0, DDG_ERR_NOT_SPD, "non-positive diagonal in row " + std::to_string(i));
        continue;
      }
      const int32_t* b = ci + rp[c];
      const int32_t* e = ci + rp[c + 1];
      const int64_t u = rp[c] + (std::lower_bound(b, e, (int32_t)i) - b);
      DDG_REQUIRE(std::fabs(val[t] - val[u]) <= 1e-14 * amax, DDG_ERR_INVALID_ARG,
                  "matrix not symmetric at (" + std::to_string(i) + "," + std::to_string(c) + ")");
    }
  }
}

// Envelope of each local matrix in its local order: per local row j, the
// columns from its first stored lower entry to j (the storage of a banded or
// envelope Cholesky factor, where the fill stays).  Also the rows of every
// expanded set with its one-ring of neighbours in the graph of A.
void count_envelope(Handle& h, const int64_t* rp, const int32_t* ci) {
  const Symbolic& S = h.S;
  std::vector<int32_t> loc((size_t)S.n, -1), stamp((size_t)S.n, -1);
  int64_t env = 0, nbhd = 0;
  for (int32_t i = 0; i < S.n_parts; ++i) {
    const int64_t r0 = S.set_ptr[i], r1 = S.set_ptr[i + 1];
    for (int64_t t = r0; t < r1; ++t) loc[S.set_idx[t]] = (int32_t)(t - r0);
    for (int64_t t = r0; t < r1; ++t) {
      const int32_t g = S.set_idx[t], j = (int32_t)(t - r0);
      int32_t first = j;
      for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
        const int32_t l = loc[ci[e]];
        if (l >= 0 && l < first) first = l;
        if (stamp[ci[e]] != i) {
          stamp[ci[e]] = i;
          ++nbhd;
        }
      }
      env += j - first + 1;
    }
    for (int64_t t = r0; t < r1; ++t) loc[S.set_idx[t]] = -1;
  }
  h.info.envelope_elems = env;
  h.info.set_rows = S.set_ptr[S.n_parts];
  h.info.nbhd_rows = nbhd;
}

// Algorithmic HBM bytes of one local-solve kernel launch per colour: factor
// tiles read once per substitution (every level twice, the middle level once),
// the couplings (ELL slots or sliced entries), and per local row the residual
// read, the set index and the read-modify-write of e in the scatter.  The
// local-residual kernel that precedes it is counted separately (residual_bytes):
// set index, r, residual write, and for colours that start from a non-zero e the
// row pointers, the CSR rows and one read of e per entry.
void account_bytes(Handle& h, const int64_t* rp, const int32_t* ci) {
  const Symbolic& S = h.S;
  const int es = storage_size(h.opt.precision);
  const int32_t C = S.n_colours;
  h.colour_bytes.assign(2 * C, 0);
  h.colour_bytes_sys.assign((size_t)h.nb * 2 * C, 0);
  h.flow_bytes_sys.assign((size_t)h.nb * 2, 0);
  std::vector<int32_t> sys_of(S.n_parts, 0);
  for (int32_t b = 0; b < h.nb; ++b)
    for (int32_t i = h.sub_off[b]; i < h.sub_off[b + 1]; ++i) sys_of[i] = b;
  int64_t resid = 0, resid0 = 0, flow0 = 0, flow1 = 0;
  for (int32_t c = 0; c < C; ++c) {
    int64_t bytes = 0;
    for (int32_t q = S.colour_ptr[c]; q < S.colour_ptr[c + 1]; ++q) {
      const int32_t i = S.colour_subs[q];
      const int64_t before = bytes, f0 = flow0, f1 = flow1;
      int64_t fb = 0;
      const int32_t K = S.sub_blk_ptr[i + 1] - S.sub_blk_ptr[i];
      for (int32_t k = 0; k < K; ++k) {
        // every level's inverse is read on the way down and back, the middle one once
        const int64_t tb = tile_bytes(S.blk_size[S.sub_blk_ptr[i] + k], S.tile, es);
        fb += tb * (k == S.sub_mid[i] ? 1 : 2);
      }
      const int64_t r0 = S.set_ptr[i], r1 = S.set_ptr[i + 1];
      const int64_t ni = r1 - r0;
      // couplings read by the local solves: ELL slots (8-byte values) or sliced entries
      // (values in the solve's arithmetic type)
      int64_t cpl = ni * (S.cl + S.cu) * 12;
      if (S.sliced) {
        const int32_t a0 = S.blk_slice[S.sub_blk_ptr[i]], a1 = S.blk_slice[S.sub_blk_ptr[i + 1]];
        const int64_t ent = (S.sl_lo_off[a1] - S.sl_lo_off[a0]) + (S.sl_up_off[a1] - S.sl_up_off[a0]);
        cpl = ent * (4 + (h.opt.precision == DDG_FP64 ? 8 : 4));
      }
      int64_t nnz_rows = 0;
      for (int64_t t = r0; t < r1; ++t) nnz_rows += rp[S.set_idx[t] + 1] - rp[S.set_idx[t]];
      if (h.ssor) {
        // SSOR: residual read, set index, e read-modify-write once; per relaxation of a
        // row (2 per sweep) its row pointer, local entries (column + value), diagonal and
        // place in the colour order; the iterate itself stays on chip
        fb = 0;
        cpl = 2 * (int64_t)h.opt.ssor_sweeps * (ni * (8 + 8 + 4) + h.ss_nnz_sub[i] * 12);
      }
      bytes += fb + cpl + ni * (8 + 4 + 16);
      resid0 += ni * (4 + 8 + 8);
      // a gathered row from the diagonals reads its diagonal and both sides' entries
      resid += ni * (4 + 8 + 8 + 8) + (h.dia_ok ? ni * 8 * (1 + 2 * (int64_t)h.dia_nd) : nnz_rows * 12 + ni * 16);
      // persistent sweep: the same local solves, each forming its residual rows itself
      // (set index, r, row pointers, CSR rows and e; set index and r when e = 0)
      const int64_t own = fb + cpl + ni * (4 + 16);
      flow1 += own + ni * (4 + 8 + 16 + 8) + nnz_rows * 12;
      flow0 += own + (c == 0 ? ni * (4 + 8) : ni * (4 + 8 + 16 + 8) + nnz_rows * 12);
      const size_t b = (size_t)sys_of[i];
      h.colour_bytes_sys[b * 2 * C + c] += bytes - before;
      h.colour_bytes_sys[b * 2 * C + C + c] += bytes - before;
      h.flow_bytes_sys[b * 2] += flow0 - f0;
      h.flow_bytes_sys[b * 2 + 1] += flow1 - f1;
    }
    h.colour_bytes[c] = bytes;
    h.colour_bytes[C + c] = bytes;
  }
  count_envelope(h, rp, ci);
  h.residual_bytes = resid;
  h.flow_bytes[0] = flow0;
  h.flow_bytes[1] = flow1;
  int64_t sweep = 0;
  if (h.flow_ok) {
    sweep = flow0 + flow1;
  } else {
    for (int32_t c = 0; c < C; ++c) sweep += 2 * h.colour_bytes[c];
    sweep += (2 * C - 1) * (resid / C) + resid0 / C;  // residual kernels (per-colour average)
  }
  h.info.sweep_bytes = sweep;
  // one full pass over A: CSR (row pointers, columns, values) or the stored diagonals
  const int64_t n = S.n, nnzb = h.dia_ok ? n * 8 * (1 + (int64_t)h.dia_nd) : S.nnz * 12 + (n + 1) * 8;
  const int64_t ntiles = h.ntiles;
  // coarse: restrict (residual SpMV + Q), tiled inverse GEMV, prolong (Q, e rmw)
  // (the dense inverse's tiles, or one application of the coarse level's preconditioner;
  // the inexact coarse solve's bytes depend on its inner iteration count: not counted)
  const int64_t core = h.inner ? h.inner->apply_bytes : h.ic ? 0 : ntiles * 64 * 64 * 8;
  const int64_t coarse = h.nc ? (nnzb + 3 * n * 8 + n * h.k * 8 + core + n * h.k * 8 + 16 * n) : 0;
  h.apply_bytes = sweep + coarse;
  // CG: SpMV (p, q), x/r/p/q update, two dots, p update
  const int64_t cg = nnzb + 2 * n * 8 + 6 * n * 8 + 4 * n * 8 + 3 * n * 8;
  h.info.iter_bytes = sweep + coarse + cg + n * 8;
  h.info.tile = S.tile;
  h.info.schedule = h.persist ? DDG_SCHEDULE_PERSISTENT : h.flow_ok ? DDG_SCHEDULE_QUEUE : DDG_SCHEDULE_COLOURS;
  h.info.factor_bytes = h.ssor ? 0 : S.fac_elems * es;
  h.info.coarse_bytes = h.nc && !h.ic ? ntiles * 64 * 64 * 8 : 0;
}

void check_err_flag(Handle& h, const char* what) {
  int32_t e[4];
  DDG_HIP(hipMemcpyAsync(e, h.err_flag.p, sizeof(e), hipMemcpyDeviceToHost, h.stream));
  DDG_HIP(hipStreamSynchronize(h.stream));
  if (e[0] != 0) {
    std::string m = std::string(what) + ": ";
    if (e[0] == DDG_ERR_RANK) m += "every generating vector vanishes on subdomain " + std::to_string(e[1]);
    else if (e[0] == DDG_ERR_HIP && e[2] == -8) m += "sweep task of subdomain " + std::to_string(e[1]) + " timed out waiting for a dependency";
    else if (e[0] == DDG_ERR_HIP && e[2] == -9) m += "sweep task queue out of step";
    else if (e[0] == DDG_ERR_HIP && e[2] == -10) m += "persistent solve: a workgroup waited too long for its next task";
    else if (e[0] == DDG_ERR_HIP && e[2] == -11) m += "grouped sweep barrier timed out in subdomain " + std::to_string(e[1]);
    else if (e[0] == DDG_ERR_HIP) m += "workgroup handoff timed out in subdomain " + std::to_string(e[1]);
    else if (e[1] < 0) m += "coarse pivot " + std::to_string(e[3]) + " not positive (A0 not SPD)";
    else m += "local pivot not positive in subdomain " + std::to_string(e[1]) + " block " + std::to_string(e[2]) +
              " row " + std::to_string(e[3]);
    DDG_HIP(hipMemsetAsync(h.err_flag.p, 0, sizeof(e), h.stream));
    if (h.twisted_ok) {
      // a partner that arrived after its handoff wait gave up has raised its flag:
      // clear every flag so that the next launch's readers wait for fresh data
      DDG_HIP(hipMemsetAsync(h.flags.p, 0, (size_t)h.S.n_parts * 2 * h.grp_max * sizeof(int32_t), h.stream));
    }
    if (h.grp_max > 1) {
      // likewise the grouped sweep's barrier counts
      DDG_HIP(hipMemsetAsync(h.gcnt.p, 0, (size_t)h.grp_slots * 2 * sizeof(int32_t), h.stream));
    }
    if (h.flow_ok) {
      // the task queue may be out of step after a failed sweep: start it afresh
      DDG_HIP(hipMemsetAsync(h.flow_done.p, 0, (size_t)h.S.n_parts * sizeof(int32_t), h.stream));
      DDG_HIP(hipMemsetAsync(h.flow_counter.p, 0, sizeof(unsigned long long), h.stream));
      h.flow_base = 0;
      h.flow_seq = 0;
    }
    throw Error{e[0], m};
  }
}

// Local CSR, diagonal positions and local colouring of every A_i for SSOR
// smoothing (integers only): colour(r) is the smallest colour not taken by a
// coupled local row r' < r, and the rows of a subdomain are listed colour by
// colour, ascending within a colour.
void build_ssor(Handle& h, const int64_t* rp, const int32_t* ci) {
  const Symbolic& S = h.S;
  const int64_t tot = S.set_ptr[S.n_parts];
  std::vector<int64_t> ptr((size_t)tot + 1, 0), pos, dpos((size_t)tot, -1);
  std::vector<int32_t> col, perm((size_t)tot), cptr((size_t)S.n_parts + 1, 0), coff;
  std::vector<int32_t> loc((size_t)S.n, -1), colour;
  h.ss_nnz_sub.assign(S.n_parts, 0);
  for (int32_t i = 0; i < S.n_parts; ++i) {
    const int64_t r0 = S.set_ptr[i], r1 = S.set_ptr[i + 1];
    const int32_t ni = (int32_t)(r1 - r0);
    for (int64_t t = r0; t < r1; ++t) loc[S.set_idx[t]] = (int32_t)(t - r0);
    colour.assign(ni, -1);
    int32_t ncol = 0;
    std::vector<char> used;
    for (int64_t t = r0; t < r1; ++t) {
      const int32_t g = S.set_idx[t], r = (int32_t)(t - r0);
      used.assign((size_t)ncol + 1, 0);
      for (int64_t e = rp[g]; e < rp[g + 1]; ++e) {
        const int32_t l = loc[ci[e]];
        if (l < 0) continue;
        col.push_back(l);
        pos.push_back(e);
        if (l == r) dpos[(size_t)t] = e;
        if (l < r) used[(size_t)colour[l]] = 1;
      }
      int32_t c = 0;
      while (used[(size_t)c]) ++c;
      colour[r] = c;
      ncol = std::max(ncol, c + 1);
      ptr[(size_t)t + 1] = (int64_t)col.size();
      DDG_REQUIRE(dpos[(size_t)t] >= 0, DDG_ERR_INVALID_ARG, "row without a stored diagonal");
    }
    h.ss_nnz_sub[i] = ptr[(size_t)r1] - ptr[(size_t)r0];
    cptr[i] = (int32_t)coff.size();
    int32_t k = 0;
    for (int32_t c = 0; c < ncol; ++c) {
      coff.push_back(k);
      for (int32_t r = 0; r < ni; ++r)
        if (colour[r] == c) perm[(size_t)(r0 + k++)] = r;
    }
    coff.push_back(k);
    for (int64_t t = r0; t < r1; ++t) loc[S.set_idx[t]] = -1;
  }
  cptr[S.n_parts] = (int32_t)coff.size();
  hipStream_t s = h.stream;
  h.ss_ptr.upload(ptr, s);
  h.ss_col.upload(col, s);
  h.ss_pos.upload(pos, s);
  h.ss_dpos.upload(dpos, s);
  h.ss_perm.upload(perm, s);
  h.ss_cptr.upload(cptr, s);
  h.ss_coff.upload(coff, s);
  h.ss_val.alloc(std::max<size_t>(1, pos.size()) * sizeof(double));
  h.ss_diag.alloc((size_t)std::max<int64_t>(1, tot) * sizeof(double));
}

void numeric_setup(Handle& h) {
  hipEvent_t e0, e1;
  DDG_HIP(hipEventCreate(&e0));
  DDG_HIP(hipEventCreate(&e1));
  DDG_HIP(hipEventRecord(e0, h.stream));
  launch_refresh_couplings(h, h.stream);
  launch_dia_refresh(h, h.stream);
  if (h.nc > 0) launch_galerkin(h, h.stream);
  // The local factorisation (wide batched launches) and the coarse inverse (a tree of
  // small, latency-bound launches) are independent: the coarse inverse runs on a
  // second stream once A0 is formed, the local levels on the handle's stream.
  hipEvent_t eg = nullptr, ec = nullptr;
  if (h.nc > 0) {
    if (!h.side) DDG_HIP(hipStreamCreateWithFlags(&h.side, hipStreamNonBlocking));
    DDG_HIP(hipEventCreateWithFlags(&eg, hipEventDisableTiming));
    DDG_HIP(hipEventCreateWithFlags(&ec, hipEventDisableTiming));
    DDG_HIP(hipEventRecord(eg, h.stream));
  }
  // the coarse chain (inverse and its accuracy measurement, or the incomplete factor)
  // is enqueued first on the side stream: it is the longer one, and its host code
  // never waits, so the local factorisation's launches follow at once
  if (h.nc > 0 && !h.three_level) {
    DDG_HIP(hipStreamWaitEvent(h.side, eg, 0));
    if (h.ic) {
      launch_ic_factor(h, h.side);
    } else {
      launch_coarse_invert(h, h.side);
      launch_coarse_measure(h, h.side);
    }
    DDG_HIP(hipEventRecord(ec, h.side));
  }
  if (h.ssor) {
    launch_gather(h.ss_pos.as<int64_t>(), h.val.as<double>(), h.ss_val.as<double>(),
                  (int64_t)(h.ss_pos.bytes / sizeof(int64_t)), h.stream);
    launch_gather(h.ss_dpos.as<int64_t>(), h.val.as<double>(), h.ss_diag.as<double>(), h.S.set_ptr[h.S.n_parts],
                  h.stream);
  } else {
    launch_local_factor(h, h.stream);
  }
  if (h.nc > 0 && !h.three_level) DDG_HIP(hipStreamWaitEvent(h.stream, ec, 0));
  if (eg) (void)hipEventDestroy(eg);
  if (ec) (void)hipEventDestroy(ec);
  if (h.inner) {
    // the coarse level's values from the new A0, then its own factorisation
    launch_gather(h.a0_pos.as<int64_t>(), h.A0.as<double>(), h.inner->val.as<double>(), h.inner->S.nnz, h.stream);
    numeric_setup(*h.inner);
  }
  DDG_HIP(hipEventRecord(e1, h.stream));
  DDG_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  DDG_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h.info.setup_ms = ms;
  check_err_flag(h, "numeric factorisation");
  if (h.nc > 0 && !h.three_level && !h.ic) {
    // accuracy of the explicit coarse inverse X: e estimates the spectral radius of
    // I - X A0; when it is not at working precision (ill-conditioned A0, e.g. the
    // biharmonic operator at large sizes), each coarse solve takes iterative-refinement
    // steps y += X (b0 - A0 y), which reduce the error by e per step and keep the coarse
    // operator symmetric (after s steps it is (I - (I - X A0)^{s+1}) A0^{-1})
    const double e = finish_coarse_measure(h);
    h.coarse_inv_err = e;
    int32_t steps = 0;
    if (!(e <= 1e-12)) {
      DDG_REQUIRE(e < 0.5, DDG_ERR_NOT_SPD,
                  "coarse inverse too inaccurate to refine (||v - X A0 v|| / ||v|| = " + std::to_string(e) + ")");
      steps = (int32_t)std::ceil(std::log(1e-13) / std::log(e)) - 1;
      steps = std::max(1, std::min(4, steps));
      if (!h.cref.p) h.cref.alloc((size_t)2 * h.nc_pad * sizeof(double));
    }
    h.coarse_refine = steps;
    h.ws.cref = h.cref.p ? h.cref.as<double>() : nullptr;
  }
  if (h.dia_possible) {
    // the diagonals represent A only when its values are symmetric bit for bit;
    // otherwise the row dots read the CSR rows (until a refactor makes them so)
    int32_t bad = 0;
    DDG_HIP(hipMemcpyAsync(&bad, h.err_flag.as<int32_t>() + 4, sizeof(bad), hipMemcpyDeviceToHost, h.stream));
    DDG_HIP(hipStreamSynchronize(h.stream));
    if (bad) DDG_HIP(hipMemsetAsync(h.err_flag.as<int32_t>() + 4, 0, sizeof(int32_t), h.stream));
    h.dia_ok = bad == 0;
  }
  h.info.matrix_format = h.dia_ok ? DDG_MATRIX_DIA : DDG_MATRIX_CSR;
  h.info.coarse_refine = h.coarse_refine;
  h.info.coarse_inverse_err = h.coarse_inv_err;
  h.info.coarse_solver = h.ic ? DDG_COARSE_IC_CG : DDG_COARSE_INVERSE;
}

// Diagonal storage is possible when no system's rows have more than kDiaMax
// distinct positive column offsets (up to 13-point stencils); the row dots then
// take one lane per row.
void plan_dia(Handle& h, const int64_t* rp, const int32_t* ci) {
  h.dia_possible = false;
  h.dia_ok = false;
  if (h.opt.matrix_format == DDG_MATRIX_CSR || std::getenv("DDG_ROW_LANES")) return;
  if (h.S.nnz > (2 * kDiaMax + 1) * h.S.n) return;
  std::vector<DiaSys> sys((size_t)h.nb);
  for (int32_t b = 0; b < h.nb; ++b) {
    DiaSys& d = sys[b];
    std::memset(&d, 0, sizeof(d));
    d.lo = h.seg_off[b];
    d.hi = h.seg_off[b + 1];
    std::vector<int32_t> offs;
    for (int64_t g = d.lo; g < d.hi; ++g) {
      for (int64_t t = rp[g]; t < rp[g + 1]; ++t) {
        const int64_t o = (int64_t)ci[t] - g;
        if (o <= 0) continue;
        if (std::find(offs.begin(), offs.end(), (int32_t)o) == offs.end()) {
          if ((int)offs.size() == kDiaMax) return;
          offs.push_back((int32_t)o);
        }
      }
    }
    std::sort(offs.begin(), offs.end());
    d.nd = (int32_t)offs.size();
    for (int32_t q = 0; q < d.nd; ++q) d.off[q] = offs[q];
  }
  int32_t nd = 0;
  for (const auto& d : sys) nd = std::max(nd, d.nd);
  h.dia_sys_h = sys;
  h.dia_nd = std::max(nd, 1);
  h.dia_sys.upload(sys, h.stream);
  h.dia_diag.alloc((size_t)h.S.n * sizeof(double));
  h.dia_up.alloc((size_t)h.dia_nd * h.S.n * sizeof(double));
  h.dia_possible = true;
  h.lpr = 1;
}

// Durations of the profiled local-solve launches.  A launch enqueued by CG
// iteration t ran for system b unless b had already stopped after at most t
// iterations (its kernels then return at once); launches outside a solve (tag
// -1) ran for every system.  Only the bytes of the systems a launch ran for are
// credited, and launches that ran for none are kept apart as idle.  The host
// mirror of the CG states must be current (it is after every convergence check).
void flush_profile(Handle& h) {
  if (h.pending.empty()) return;
  DDG_HIP(hipStreamSynchronize(h.stream));
  const int32_t C = h.S.n_colours;
  for (auto& pl : h.pending) {
    float ms = 0.f;
    DDG_HIP(hipEventElapsedTime(&ms, h.ev_pool[pl.ev], h.ev_pool[pl.ev + 1]));
    int64_t bytes = 0;
    for (int32_t b = 0; b < h.nb; ++b) {
      const CgState& st = h.h_state[b];
      const bool ran = pl.tag < 0 || !st.done || st.iters > pl.tag;
      if (!ran) continue;
      bytes += pl.what < 2 * C ? h.colour_bytes_sys[(size_t)b * 2 * C + pl.what]
                               : h.flow_bytes_sys[(size_t)b * 2 + (pl.what - 2 * C)];
    }
    if (bytes > 0) {
      h.prof_ms += ms;
      h.prof_launches += 1;
      h.prof_bytes += bytes;
    } else {
      h.prof_idle_ms += ms;
      h.prof_idle_launches += 1;
    }
  }
  h.pending.clear();
  h.ev_used = 0;
}

// Smallest and largest eigenvalue of the symmetric tridiagonal matrix (d, e)
// (e[j] couples rows j and j+1) by bisection on the Sturm count.
void tridiag_extremes(const std::vector<double>& d, const std::vector<double>& e, double& lo, double& hi) {
  const size_t m = d.size();
  double gl = d[0], gu = d[0];
  for (size_t j = 0; j < m; ++j) {
    const double r = (j > 0 ? std::fabs(e[j - 1]) : 0.0) + (j + 1 < m ? std::fabs(e[j]) : 0.0);
    gl = std::min(gl, d[j] - r);
    gu = std::max(gu, d[j] + r);
  }
  auto below = [&](double x) {  // eigenvalues < x
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (size_t j = 1; j < m; ++j) {
      if (q == 0.0) q = 1e-300;
      q = d[j] - x - e[j - 1] * e[j - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  auto kth = [&](int k) {  // smallest x with below(x) >= k
    double a = gl, b = gu;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double mid = 0.5 * (a + b);
      if (below(mid) >= k) b = mid;
      else a = mid;
    }
    return 0.5 * (a + b);
  };
  lo = kth(1);
  hi = kth((int)m);
}

// Setup of one handle holding nb independent systems: system b owns rows
// [seg_off[b], seg_off[b+1]) and subdomains [sub_off[b], sub_off[b+1]); the
// matrix has no entries between systems.
void setup_impl(Handle& hh, int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val,
                int32_t k, const double* F, const int32_t* part, int32_t n_parts, int32_t overlap,
                const std::vector<int64_t>& seg_off, const std::vector<int32_t>& sub_off) {
  Handle* h = &hh;
  if (h->opt.max_iter <= 0) h->opt.max_iter = 1000;
  if (h->opt.check_every <= 0) h->opt.check_every = 4;
  DDG_REQUIRE(h->opt.precision >= DDG_FP64 && h->opt.precision <= DDG_MIXED_BF16, DDG_ERR_INVALID_ARG,
              "unknown precision");
  DDG_REQUIRE(h->opt.rtol >= 0.0 && h->opt.rank_tol >= 0.0, DDG_ERR_INVALID_ARG, "negative tolerance");
  DDG_REQUIRE(h->opt.cg_variant == DDG_CG_FLETCHER_REEVES || h->opt.cg_variant == DDG_CG_POLAK_RIBIERE,
              DDG_ERR_INVALID_ARG, "cg_variant must be a ddg_cg_variant value");
  DDG_REQUIRE(h->opt.local_solver == DDG_LOCAL_EXACT || h->opt.local_solver == DDG_LOCAL_SSOR,
              DDG_ERR_INVALID_ARG, "local_solver must be a ddg_local_solver value");
  DDG_REQUIRE(h->opt.coarse_solver == DDG_COARSE_INVERSE || h->opt.coarse_solver == DDG_COARSE_IC_CG,
              DDG_ERR_INVALID_ARG, "coarse_solver must be a ddg_coarse_solver value");
  h->ic = h->opt.coarse_solver == DDG_COARSE_IC_CG;
  if (h->ic) {
    DDG_REQUIRE(h->opt.ic_tol >= 0.0 && h->opt.ic_maxit >= 1, DDG_ERR_INVALID_ARG,
                "the incomplete Cholesky coarse solve needs ic_tol >= 0 and ic_maxit >= 1");
    DDG_REQUIRE(!h->three_level, DDG_ERR_UNSUPPORTED,
                "the three-level cycle replaces the coarse solve; use DDG_COARSE_INVERSE with it");
  }
  h->ssor = h->opt.local_solver == DDG_LOCAL_SSOR;
  if (h->ssor)
    DDG_REQUIRE(h->opt.ssor_omega > 0.0 && h->opt.ssor_omega < 2.0 && h->opt.ssor_sweeps >= 1, DDG_ERR_INVALID_ARG,
                "SSOR needs 0 < ssor_omega < 2 and ssor_sweeps >= 1");
  h->stream = static_cast<hipStream_t>(h->opt.stream);
  h->k = k;
  h->nb = (int32_t)seg_off.size() - 1;
  h->seg_off = seg_off;
  h->sub_off = sub_off;
  DDG_REQUIRE(k <= kMaxGen, DDG_ERR_UNSUPPORTED, "at most 80 generating vectors");
  if (k > 0)
    for (int64_t t = 0; t < n * (int64_t)k; ++t)
      DDG_REQUIRE(std::isfinite(F[t]), DDG_ERR_INVALID_ARG, "non-finite generating vectors");
  build_symbolic(h->S, n, row_ptr, col_idx, part, n_parts, overlap, h->opt.tile, h->opt.block_target);
  check_values(n, row_ptr, col_idx, val);
  Symbolic& S = h->S;
  int dev = 0;
  DDG_HIP(hipGetDevice(&dev));
  h->device = dev;
  int lds = 0;
  DDG_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  h->dev_lds_limit = lds;
  int clk = 0;
  DDG_HIP(hipDeviceGetAttribute(&clk, hipDeviceAttributeWallClockRate, dev));
  h->clock_khz = clk > 0 ? clk : 100000;
  hipStream_t s = h->stream;
  // system of each subdomain
  std::vector<int32_t> si(n_parts, 0);
  for (int32_t b = 0; b < h->nb; ++b)
    for (int32_t i = sub_off[b]; i < sub_off[b + 1]; ++i) si[i] = b;
  h->sub_inst.upload(si, s);
  // integer structure
  std::vector<int64_t> rp(row_ptr, row_ptr + n + 1);
  std::vector<int32_t> ci(col_idx, col_idx + S.nnz);
  std::vector<double> vv(val, val + S.nnz);
  std::vector<int32_t> pp(part, part + n);
  h->rowptr.upload(rp, s);
  h->col.upload(ci, s);
  h->val.upload(vv, s);
  h->part.upload(pp, s);
  h->own_ptr.upload(S.own_ptr, s);
  h->own_idx.upload(S.own_idx, s);
  h->set_ptr.upload(S.set_ptr, s);
  h->set_idx.upload(S.set_idx, s);
  h->colour_subs.upload(S.colour_subs, s);
  h->nbr_ptr.upload(S.nbr_ptr, s);
  h->nbr_idx.upload(S.nbr_idx, s);
  h->sub_blk_ptr.upload(S.sub_blk_ptr, s);
  h->blk_start.upload(S.blk_start, s);
  h->blk_size.upload(S.blk_size, s);
  h->blk_foff.upload(S.blk_foff, s);
  h->sub_mid.upload(S.sub_mid, s);
  h->lo_col.upload(S.lo_col, s);
  h->lo_pos.upload(S.lo_pos, s);
  h->up_col.upload(S.up_col, s);
  h->up_pos.upload(S.up_pos, s);
  h->in_ptr.upload(S.in_ptr, s);
  h->in_col.upload(S.in_col, s);
  h->in_pos.upload(S.in_pos, s);
  h->lo_val.alloc(std::max<size_t>(1, S.lo_pos.size()) * sizeof(double));
  h->up_val.alloc(std::max<size_t>(1, S.up_pos.size()) * sizeof(double));
  if (S.sliced) {
    h->blk_slice.upload(S.blk_slice, s);
    h->sl_row.upload(S.sl_row, s);
    h->sl_rows.upload(S.sl_rows, s);
    h->sl_lo_off.upload(S.sl_lo_off, s);
    h->sl_up_off.upload(S.sl_up_off, s);
    h->sl_lo_col.upload(S.sl_lo_col, s);
    h->sl_up_col.upload(S.sl_up_col, s);
    const size_t vs = h->opt.precision == DDG_FP64 ? sizeof(double) : sizeof(float);
    h->sl_lo_val.alloc(std::max<size_t>(1, S.sl_lo_col.size()) * vs);
    h->sl_up_val.alloc(std::max<size_t>(1, S.sl_up_col.size()) * vs);
  }
  // two-workgroup sweep: every pair of a colour must be resident at once
  int ncu = 0;
  DDG_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  h->n_cu = ncu;
  int max_nsub = 0;
  for (int32_t c = 0; c < S.n_colours; ++c) max_nsub = std::max(max_nsub, S.colour_ptr[c + 1] - S.colour_ptr[c]);
  h->twisted_ok = (16 * ((max_nsub + 7) / 8) <= ncu) && std::getenv("DDG_NO_TWIST") == nullptr;
  h->xch_ld = ((S.max_blk + 63) / 64) * 64;
  // grouped sweep: with the sliced coupling layout (wide levels), when a colour leaves
  // CUs idle; DDG_SWEEP_GROUPS caps the group size (1 = off), DDG_SWEEP_SPLIT_ROUNDS
  // sets the narrowest split level in rounds
  if (S.sliced && h->opt.local_solver == DDG_LOCAL_EXACT) {
    h->grp_max = kSweepGroupsMax;
    if (const char* env = std::getenv("DDG_SWEEP_GROUPS")) h->grp_max = std::max(1, std::min(kSweepGroupsCap, std::atoi(env)));
    h->grp_split = kSweepSplitRounds;
    if (const char* env = std::getenv("DDG_SWEEP_SPLIT_ROUNDS")) h->grp_split = std::max(2, std::atoi(env));
  }
  if (h->grp_max > 1) {
    h->grp_slots = max_nsub;
    h->gx.alloc((size_t)max_nsub * 2 * 2 * h->grp_max * h->xch_ld * sizeof(double));
    h->gcnt.alloc((size_t)max_nsub * 2 * sizeof(int32_t));
    DDG_HIP(hipMemsetAsync(h->gcnt.p, 0, (size_t)max_nsub * 2 * sizeof(int32_t), s));
  }
  if (h->twisted_ok) {
    h->xch.alloc((size_t)n_parts * 2 * h->xch_ld * sizeof(double));
    h->flags.alloc((size_t)n_parts * 2 * h->grp_max * sizeof(int32_t));
    DDG_HIP(hipMemsetAsync(h->flags.p, 0, (size_t)n_parts * 2 * h->grp_max * sizeof(int32_t), s));
  }
  h->bres.alloc((size_t)S.set_ptr[n_parts] * sizeof(double));
  // [0..3] setup/solve error (code, subdomain, block, pivot); [4] entries whose transpose
  // differs in its bits (diagonal storage check)
  h->err_flag.alloc(8 * sizeof(int32_t));
  DDG_HIP(hipMemsetAsync(h->err_flag.p, 0, 8 * sizeof(int32_t), s));
  // (SSOR smoothing stores no local factors)
  h->fac.alloc(h->ssor ? 16 : (size_t)S.fac_elems * storage_size(h->opt.precision));
  if (h->ssor) build_ssor(*h, row_ptr, col_idx);
  // coarse basis (depends only on F and the partition)
  h->kcnt.assign(n_parts, 0);
  h->koff.assign(n_parts + 1, 0);
  h->cblk_off.assign(h->nb + 1, 0);
  h->cblk_n.assign(h->nb, 0);
  if (k > 0) {
    h->F.alloc((size_t)n * k * sizeof(double));
    DDG_HIP(hipMemcpyAsync(h->F.p, F, (size_t)n * k * sizeof(double), hipMemcpyHostToDevice, s));
    h->Q.alloc((size_t)n * k * sizeof(double));
    h->kcnt_d.alloc((size_t)n_parts * sizeof(int32_t));
    launch_coarse_basis(*h, s);
    check_err_flag(*h, "coarse basis");
    launch_q_own(*h, s);
    DDG_HIP(hipMemcpyAsync(h->kcnt.data(), h->kcnt_d.p, (size_t)n_parts * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s));
    DDG_HIP(hipStreamSynchronize(s));
    // coarse numbering: subdomain order, each system's block padded to a multiple of 64
    int64_t run = 0;
    for (int32_t b = 0; b < h->nb; ++b) {
      h->cblk_off[b] = run;
      for (int32_t i = sub_off[b]; i < sub_off[b + 1]; ++i) {
        h->koff[i] = run;
        run += h->kcnt[i];
      }
      h->cblk_n[b] = (int32_t)(run - h->cblk_off[b]);
      h->nc += h->cblk_n[b];
      run = (run + 63) / 64 * 64;
    }
    h->koff[n_parts] = run;
    h->cblk_off[h->nb] = run;
    h->koff_d.upload(h->koff, s);
    if (!h->three_level) h->F.release();   // a three-level handle still forms F0 = R0 F
  }
  h->nc_pad = h->cblk_off[h->nb];
  if (h->nc > 0) {
    h->a0_off.assign(h->nb + 1, 0);
    h->tile_base.assign(h->nb + 1, 0);
    std::vector<int32_t> tinst, rinst;
    for (int32_t b = 0; b < h->nb; ++b) {
      const int64_t nbk = h->cblk_n[b];
      const int64_t ntr = (h->cblk_off[b + 1] - h->cblk_off[b]) / 64;
      h->a0_off[b + 1] = h->a0_off[b] + nbk * nbk;
      h->tile_base[b + 1] = h->tile_base[b] + ntr * (ntr + 1) / 2;
      tinst.insert(tinst.end(), (size_t)(ntr * (ntr + 1) / 2), b);
      rinst.insert(rinst.end(), (size_t)ntr, b);
    }
    h->ntiles = h->tile_base[h->nb];
    h->cblk_off_d.upload(h->cblk_off, s);
    h->cblk_n_d.upload(h->cblk_n, s);
    h->a0_off_d.upload(h->a0_off, s);
    h->tile_base_d.upload(h->tile_base, s);
    h->tile_inst.upload(tinst, s);
    h->trow_inst.upload(rinst, s);
    h->A0.alloc((size_t)h->a0_off[h->nb] * sizeof(double));
    if (!h->three_level && !h->ic) h->A0inv_t.alloc((size_t)h->ntiles * 64 * 64 * sizeof(double));
    h->cy.alloc((size_t)2 * h->nc_pad * sizeof(double));
    DDG_HIP(hipMemsetAsync(h->cy.p, 0, (size_t)2 * h->nc_pad * sizeof(double), s));
    if (!h->three_level && !h->ic) h->cpart.alloc((size_t)2 * h->ntiles * 64 * sizeof(double));
  }
  // row-dot kernels: lanes per CSR row; the coarse restriction runs four passes of
  // its workgroup per chunk of own rows
  h->lpr = lanes_per_row(S.nnz, n);
  if (const char* env = std::getenv("DDG_ROW_LANES")) {
    const int v = std::atoi(env);
    if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16) h->lpr = v;
  }
  DDG_REQUIRE(h->opt.matrix_format == DDG_MATRIX_AUTO || h->opt.matrix_format == DDG_MATRIX_CSR,
              DDG_ERR_INVALID_ARG, "matrix_format must be DDG_MATRIX_AUTO or DDG_MATRIX_CSR");
  plan_dia(*h, row_ptr, col_idx);
  // sweep over a device task queue (each task forms its own residual rows) on request;
  // the automatic choice is the colour launches (measured: 21.7 vs 21.9 ms at 128^3
  // FP32, 123 vs 139 ms for the batch of 256)
  DDG_REQUIRE(h->opt.schedule >= DDG_SCHEDULE_AUTO && h->opt.schedule <= DDG_SCHEDULE_PERSISTENT,
              DDG_ERR_INVALID_ARG, "schedule must be a ddg_schedule value");
  h->flow_ok = h->opt.schedule == DDG_SCHEDULE_QUEUE;
  DDG_REQUIRE(!(h->flow_ok && h->ssor), DDG_ERR_UNSUPPORTED, "SSOR smoothing runs with the colour launches only");
  if (h->flow_ok) {
    const int32_t C = S.n_colours;
    for (int dir = 0; dir < 2; ++dir) {
      std::vector<int32_t> order;
      order.reserve(n_parts);
      for (int32_t q = 0; q < C; ++q) {
        const int32_t c = dir == 0 ? q : C - 1 - q;
        for (int32_t t = S.colour_ptr[c]; t < S.colour_ptr[c + 1]; ++t) order.push_back(S.colour_subs[t]);
      }
      std::vector<int32_t> dptr(n_parts + 1, 0), didx;
      for (int32_t i = 0; i < n_parts; ++i) {
        for (int32_t t = S.conf_ptr[i]; t < S.conf_ptr[i + 1]; ++t) {
          const int32_t j = S.conf_idx[t];
          if (dir == 0 ? S.colour[j] < S.colour[i] : S.colour[j] > S.colour[i]) didx.push_back(j);
        }
        dptr[i + 1] = (int32_t)didx.size();
      }
      if (didx.empty()) didx.push_back(0);
      h->flow_order[dir].upload(order, s);
      h->flow_dep_ptr[dir].upload(dptr, s);
      h->flow_dep_idx[dir].upload(didx, s);
    }
    h->flow_done.alloc((size_t)n_parts * sizeof(int32_t));
    DDG_HIP(hipMemsetAsync(h->flow_done.p, 0, (size_t)n_parts * sizeof(int32_t), s));
    h->flow_counter.alloc(sizeof(unsigned long long));
    DDG_HIP(hipMemsetAsync(h->flow_counter.p, 0, sizeof(unsigned long long), s));
    h->flow_base = 0;
    h->flow_seq = 0;
  }
  h->rch = 4 * 256 / h->lpr;
  h->nch = std::max<int32_t>(1, (S.max_own + h->rch - 1) / h->rch);
  if (h->nc > 0) h->rpart.alloc((size_t)n_parts * h->nch * kslots(k) * sizeof(double));
  // CG workspace
  h->r.alloc((size_t)n * sizeof(double));
  h->p.alloc((size_t)n * sizeof(double));
  h->q.alloc((size_t)n * sizeof(double));
  h->z.alloc((size_t)n * sizeof(double));
  build_cg_map(*h, s);
  h->cstate.alloc((size_t)h->nb * sizeof(CgState));
  DDG_HIP(hipHostMalloc((void**)&h->h_state, (size_t)h->nb * sizeof(CgState), hipHostMallocDefault));
  h->sys_info.assign(h->nb, ddg_info{});
  h->ws.bres = h->bres.as<double>();
  h->ws.rpart = h->nc > 0 ? h->rpart.as<double>() : nullptr;
  h->ws.cy = h->nc > 0 ? h->cy.as<double>() : nullptr;
  h->ws.cpart = h->nc > 0 && !h->three_level && !h->ic ? h->cpart.as<double>() : nullptr;
  if (h->ic && h->nc > 0) prepare_ic(*h, s);
  h->persist = h->opt.schedule == DDG_SCHEDULE_PERSISTENT;
  if (h->persist) prepare_persist(*h, s);
  numeric_setup(*h);
  account_bytes(*h, row_ptr, col_idx);
  h->info.n_coarse = (int32_t)h->nc;
  h->info.levels = h->nc > 0 ? 2 : 1;
  h->info.n_coarsest = (int32_t)h->nc;
  h->info.n_colours = S.n_colours;
  h->info.n_parts = n_parts;
  h->info.n_blocks = (int32_t)S.blk_size.size();
}

// One block-diagonal system from the listed systems: rows, columns and
// subdomain ids shifted per system; generating vectors padded with zero
// columns up to the largest k (the rank rule drops them).
void setup_batch(Handle& h, const std::vector<const ddg_problem*>& probs, int32_t overlap) {
  const int32_t nb = (int32_t)probs.size();
  std::vector<int64_t> seg_off(nb + 1, 0);
  std::vector<int32_t> sub_off(nb + 1, 0);
  int64_t nnz = 0;
  int32_t kmax = 0;
  for (int32_t b = 0; b < nb; ++b) {
    const ddg_problem& P = *probs[b];
    DDG_REQUIRE(P.n > 0 && P.row_ptr && P.col_idx && P.val && P.part && P.n_parts > 0, DDG_ERR_INVALID_ARG,
                "system " + std::to_string(b) + ": null argument or empty");
    DDG_REQUIRE(P.k >= 0 && (P.k == 0 || P.F), DDG_ERR_INVALID_ARG,
                "system " + std::to_string(b) + ": k must be >= 0 and F given when k > 0");
    DDG_REQUIRE(P.row_ptr[0] == 0 && P.row_ptr[P.n] >= P.n, DDG_ERR_INVALID_ARG,
                "system " + std::to_string(b) + ": bad row pointers");
    seg_off[b + 1] = seg_off[b] + P.n;
    sub_off[b + 1] = sub_off[b] + P.n_parts;
    nnz += P.row_ptr[P.n];
    kmax = std::max(kmax, P.k);
  }
  const int64_t n = seg_off[nb];
  DDG_REQUIRE(n < INT32_MAX, DDG_ERR_UNSUPPORTED, "batch exceeds 2^31 - 1 rows");
  std::vector<int64_t> rp(n + 1, 0);
  std::vector<int32_t> ci((size_t)nnz);
  std::vector<double> vv((size_t)nnz);
  std::vector<int32_t> pp((size_t)n);
  std::vector<double> Fc((size_t)n * kmax, 0.0);
  for (int32_t b = 0; b < nb; ++b) {
    const ddg_problem& P = *probs[b];
    const int64_t r0 = seg_off[b], e0 = rp[r0];
    for (int64_t i = 0; i < P.n; ++i) {
      rp[r0 + i + 1] = e0 + P.row_ptr[i + 1];
      const int32_t pi = P.part[i];
      DDG_REQUIRE(pi >= 0 && pi < P.n_parts, DDG_ERR_INVALID_ARG,
                  "system " + std::to_string(b) + ": partition id out of range");
      pp[r0 + i] = pi + sub_off[b];
    }
    for (int64_t t = 0; t < P.row_ptr[P.n]; ++t) {
      const int32_t c = P.col_idx[t];
      DDG_REQUIRE(c >= 0 && c < P.n, DDG_ERR_INVALID_ARG, "system " + std::to_string(b) + ": column out of range");
      ci[e0 + t] = (int32_t)(c + r0);
      vv[e0 + t] = P.val[t];
    }
    for (int32_t m = 0; m < P.k; ++m)
      for (int64_t i = 0; i < P.n; ++i) Fc[(size_t)m * n + r0 + i] = P.F[(size_t)m * P.n + i];
  }
  setup_impl(h, n, rp.data(), ci.data(), vv.data(), kmax, kmax ? Fc.data() : nullptr, pp.data(), sub_off[nb],
             overlap, seg_off, sub_off);
}

// Autotuner of the local-solve launch shape.  Candidates: tile edge T in
// {16, 32, 64} x level merge target in {0 (merge only levels under 16 rows),
// 64, 128}.  Each candidate is set up on a sample of the batch (max_sample
// systems spread evenly over the size order; by default enough for about 4096
// subdomains, so that the launches are as full as the whole batch's) and
// timed over preconditioner applications with HIP events; the fastest is
// returned.  Results are cached by a key of the batch's shape in a text file.
std::string tune_key(int32_t nb, const ddg_problem* probs, int32_t overlap, const ddg_options& o) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      hsh ^= (v >> (8 * i)) & 0xff;
      hsh *= 1099511628211ull;
    }
  };
  mix((uint64_t)nb);
  for (int32_t b = 0; b < nb; ++b) {
    mix((uint64_t)probs[b].n);
    mix((uint64_t)probs[b].row_ptr[probs[b].n]);
    mix((uint64_t)probs[b].k);
    mix((uint64_t)probs[b].n_parts);
  }
  mix((uint64_t)overlap);
  mix((uint64_t)o.precision);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    for (const char* c = prop.gcnArchName; *c; ++c) mix((uint64_t)(unsigned char)*c);
  char buf[17];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)hsh);
  return buf;
}

void tune_batch(int32_t nb, const ddg_problem* probs, int32_t overlap, const ddg_options& base, int32_t max_sample,
                const char* cache_path, ddg_options& best, ddg_tune_entry* report, int32_t report_cap,
                int32_t* n_report) {
  best = base;
  const std::string key = tune_key(nb, probs, overlap, base);
  if (n_report) *n_report = 0;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string k;
    int32_t t, bt;
    double ms;
    while (in >> k >> t >> bt >> ms) {
      if (k == key) {
        best.tile = t;
        best.block_target = bt;
        return;
      }
    }
  }
  // sample: systems at evenly spaced positions of the size order
  std::vector<int32_t> order(nb);
  for (int32_t b = 0; b < nb; ++b) order[b] = b;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) { return probs[a].n < probs[c].n; });
  // default sample size: enough systems for about 4096 subdomains (a colour's launch then
  // has as many workgroups as the full batch would keep resident), all if fewer
  int32_t ns = max_sample;
  if (ns <= 0) {
    int64_t parts = 0;
    for (int32_t b = 0; b < nb; ++b) parts += probs[b].n_parts;
    const double avg = (double)parts / nb;
    ns = (int32_t)std::ceil(4096.0 / std::max(1.0, avg));
  }
  ns = std::max(1, std::min(ns, nb));
  std::vector<const ddg_problem*> sample;
  for (int32_t q = 0; q < ns; ++q) {
    const int32_t pos = ns == 1 ? nb - 1 : (int32_t)((int64_t)q * (nb - 1) / (ns - 1));
    if (sample.empty() || sample.back() != probs + order[pos]) sample.push_back(probs + order[pos]);
  }
  const int32_t tiles[3] = {16, 32, 64};
  const int32_t targets[3] = {0, 64, 128};
  double best_ms = -1.0;
  int32_t cnt = 0;
  for (int32_t T : tiles) {
    for (int32_t bt : targets) {
      double ms = -1.0;
      int64_t fbytes = 0;
      try {
        Handle h;
        h.opt = base;
        h.opt.tile = T;
        h.opt.block_target = bt;
        setup_batch(h, sample, overlap);
        fbytes = h.info.factor_bytes;
        const int64_t n = h.S.n;
        DevBuf r, z;
        r.alloc((size_t)n * sizeof(double));
        z.alloc((size_t)n * sizeof(double));
        launch_fill(r.as<double>(), 1.0, n, h.stream);
        launch_precond(h, r.as<double>(), z.as<double>(), -1, false, h.stream);
        hipEvent_t e0, e1;
        DDG_HIP(hipEventCreate(&e0));
        DDG_HIP(hipEventCreate(&e1));
        const int reps = 5;
        DDG_HIP(hipEventRecord(e0, h.stream));
        for (int t = 0; t < reps; ++t) launch_precond(h, r.as<double>(), z.as<double>(), -1, false, h.stream);
        DDG_HIP(hipEventRecord(e1, h.stream));
        DDG_HIP(hipEventSynchronize(e1));
        float f = 0.f;
        DDG_HIP(hipEventElapsedTime(&f, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        check_err_flag(h, "tuning");
        ms = f / reps;
        DDG_HIP(hipStreamSynchronize(h.stream));
      } catch (const Error& e) {
        if (e.code != DDG_ERR_UNSUPPORTED) throw;  // a candidate the shapes cannot use is skipped
      }
      if (report && cnt < report_cap) report[cnt] = ddg_tune_entry{T, bt, ms, fbytes};
      ++cnt;
      if (ms >= 0.0 && (best_ms < 0.0 || ms < best_ms)) {
        best_ms = ms;
        best.tile = T;
        best.block_target = bt;
      }
    }
  }
  if (n_report) *n_report = std::min(cnt, report_cap);
  DDG_REQUIRE(best_ms >= 0.0, DDG_ERR_UNSUPPORTED, "no launch shape fits the local problems");
  if (cache_path) {
    std::ofstream outf(cache_path, std::ios::app);
    outf << key << ' ' << best.tile << ' ' << best.block_target << ' ' << best_ms << '\n';
  }
}

}  // namespace

}  // namespace ddg

using namespace ddg;

extern "C" {

void ddg_default_options(ddg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = DDG_FP64;
  opt->max_iter = 1000;
  opt->rtol = 1e-8;
  opt->rank_tol = 1e-10;
  opt->tile = 0;
  opt->block_target = 0;
  opt->check_every = 4;
  opt->schedule = DDG_SCHEDULE_AUTO;
  opt->cg_variant = DDG_CG_FLETCHER_REEVES;
  opt->matrix_format = DDG_MATRIX_AUTO;
  opt->local_solver = DDG_LOCAL_EXACT;
  opt->ssor_omega = 1.0;
  opt->ssor_sweeps = 1;
  opt->coarse_solver = DDG_COARSE_INVERSE;
  opt->ic_tol = 1e-6;
  opt->ic_maxit = 200;
  opt->stream = nullptr;
}

const char* ddg_last_error(void) { return g_last_error.c_str(); }

int ddg_setup(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const double* val,
              int32_t k, const double* F, const int32_t* part, int32_t n_parts, int32_t overlap,
              const ddg_options* opt) {
  if (out) *out = nullptr;
  Handle* hp = nullptr;
  int rc = guarded([&]() {
    DDG_REQUIRE(out && row_ptr && col_idx && val && part, DDG_ERR_INVALID_ARG, "null argument");
    DDG_REQUIRE(k >= 0 && (k == 0 || F), DDG_ERR_INVALID_ARG, "k must be >= 0 and F given when k > 0");
    auto h = std::make_unique<Handle>();
    if (opt) h->opt = *opt;
    else ddg_default_options(&h->opt);
    setup_impl(*h, n, row_ptr, col_idx, val, k, F, part, n_parts, overlap, {0, n}, {0, n_parts});
    hp = h.release();
  });
  if (rc == DDG_OK) *out = reinterpret_cast<ddg_handle>(hp);
  return rc;
}

int ddg_setup_three_level(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx,
                          const double* val, int32_t k, const double* F, const int32_t* part, int32_t n_parts,
                          int32_t overlap, const int32_t* part0, int32_t n_parts0, const ddg_options* opt) {
  if (out) *out = nullptr;
  Handle* hp = nullptr;
  int rc = guarded([&]() {
    DDG_REQUIRE(out && row_ptr && col_idx && val && part && part0, DDG_ERR_INVALID_ARG, "null argument");
    DDG_REQUIRE(k > 0 && F, DDG_ERR_INVALID_ARG, "the three-level method needs generating vectors (k > 0)");
    DDG_REQUIRE(n_parts > 0 && n_parts0 > 0, DDG_ERR_INVALID_ARG, "empty partition");
    std::vector<int32_t> used(n_parts0, 0);
    for (int32_t i = 0; i < n_parts; ++i) {
      DDG_REQUIRE(part0[i] >= 0 && part0[i] < n_parts0, DDG_ERR_INVALID_ARG,
                  "coarse partition id out of range at subdomain " + std::to_string(i));
      used[part0[i]] = 1;
    }
    for (int32_t c = 0; c < n_parts0; ++c)
      DDG_REQUIRE(used[c], DDG_ERR_INVALID_ARG, "empty coarse subdomain " + std::to_string(c));
    auto h = std::make_unique<Handle>();
    if (opt) h->opt = *opt;
    else ddg_default_options(&h->opt);
    h->three_level = true;
    setup_impl(*h, n, row_ptr, col_idx, val, k, F, part, n_parts, overlap, {0, n}, {0, n_parts});
    hipStream_t s = h->stream;
    const Symbolic& S = h->S;
    const int64_t nc = h->nc;
    DDG_REQUIRE(nc > 0, DDG_ERR_RANK, "no coarse columns");
    // the coarse level's matrix: A0 with the block pattern of the subdomain couplings
    // (the unknowns of subdomains i and j are coupled when A couples their sets)
    std::vector<double> A0((size_t)(nc * nc));
    DDG_HIP(hipMemcpyAsync(A0.data(), h->A0.p, A0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    std::vector<int64_t> rp0((size_t)nc + 1, 0), pos;
    std::vector<int32_t> ci0, part_c((size_t)nc);
    for (int32_t i = 0; i < n_parts; ++i) {
      for (int32_t jj = 0; jj < h->kcnt[i]; ++jj) {
        const int64_t a = h->koff[i] + jj;
        part_c[(size_t)a] = part0[i];
        for (int32_t t = S.nbr_ptr[i]; t < S.nbr_ptr[i + 1]; ++t) {
          const int32_t j = S.nbr_idx[t];
          for (int32_t m = 0; m < h->kcnt[j]; ++m) {
            ci0.push_back((int32_t)(h->koff[j] + m));
            pos.push_back(a * nc + h->koff[j] + m);
          }
        }
        rp0[(size_t)a + 1] = (int64_t)ci0.size();
      }
    }
    // F0 = R0 F on the device
    DevBuf F0d;
    F0d.alloc((size_t)h->nc_pad * k * sizeof(double));
    launch_restrict_columns(*h, F0d.as<double>(), s);
    std::vector<double> F0((size_t)(h->nc_pad * k));
    DDG_HIP(hipMemcpyAsync(F0.data(), F0d.p, F0.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    DDG_HIP(hipStreamSynchronize(s));
    h->F.release();
    std::vector<double> F0c((size_t)(nc * k)), v0(pos.size());
    for (int32_t c = 0; c < k; ++c)
      for (int64_t a = 0; a < nc; ++a) F0c[(size_t)(c * nc + a)] = F0[(size_t)(c * h->nc_pad + a)];
    for (size_t t = 0; t < pos.size(); ++t) v0[t] = A0[(size_t)pos[t]];
    // the coarse level: FP64 throughout, colour launches, the library's tile choice
    auto in = std::make_unique<Handle>();
    in->opt = h->opt;
    in->opt.precision = DDG_FP64;
    in->opt.tile = 0;
    in->opt.block_target = 0;
    in->opt.schedule = DDG_SCHEDULE_COLOURS;
    in->opt.local_solver = DDG_LOCAL_EXACT;
    try {
      setup_impl(*in, nc, rp0.data(), ci0.data(), v0.data(), k, F0c.data(), part_c.data(), n_parts0, overlap,
                 {0, nc}, {0, n_parts0});
    } catch (Error& e) {
      e.msg = "coarse level: " + e.msg;
      throw;
    }
    h->a0_pos.upload(pos, s);
    h->inner = in.release();
    account_bytes(*h, row_ptr, col_idx);
    h->info.levels = 3;
    h->info.n_coarsest = (int32_t)h->inner->nc;
    DDG_HIP(hipStreamSynchronize(s));
    hp = h.release();
  });
  if (rc == DDG_OK) *out = reinterpret_cast<ddg_handle>(hp);
  return rc;
}

int ddg_setup_batched(ddg_handle* out, int32_t nb, const ddg_problem* probs, int32_t overlap,
                      const ddg_options* opt) {
  if (out) *out = nullptr;
  Handle* hp = nullptr;
  int rc = guarded([&]() {
    DDG_REQUIRE(out && probs && nb >= 1, DDG_ERR_INVALID_ARG, "null argument or empty batch");
    std::vector<const ddg_problem*> list(nb);
    for (int32_t b = 0; b < nb; ++b) list[b] = probs + b;
    auto h = std::make_unique<Handle>();
    if (opt) h->opt = *opt;
    else ddg_default_options(&h->opt);
    setup_batch(*h, list, overlap);
    hp = h.release();
  });
  if (rc == DDG_OK) *out = reinterpret_cast<ddg_handle>(hp);
  return rc;
}

int ddg_tune_batched(int32_t nb, const ddg_problem* probs, int32_t overlap, const ddg_options* base,
                     int32_t max_sample, const char* cache_path, ddg_options* best, ddg_tune_entry* report,
                     int32_t report_cap, int32_t* n_report) {
  return guarded([&]() {
    DDG_REQUIRE(probs && nb >= 1 && best, DDG_ERR_INVALID_ARG, "null argument or empty batch");
    ddg_options b0;
    if (base) b0 = *base;
    else ddg_default_options(&b0);
    tune_batch(nb, probs, overlap, b0, max_sample, cache_path, *best, report, report_cap, n_report);
  });
}

int ddg_analyze(ddg_handle* out, int64_t n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* part,
                int32_t n_parts, int32_t overlap, const ddg_options* opt) {
  if (out) *out = nullptr;
  Handle* hp = nullptr;
  int rc = guarded([&]() {
    DDG_REQUIRE(out && row_ptr && col_idx && part, DDG_ERR_INVALID_ARG, "null argument");
    auto h = std::make_unique<Handle>();
    if (opt) h->opt = *opt;
    else ddg_default_options(&h->opt);
    h->host_only = true;
    build_symbolic(h->S, n, row_ptr, col_idx, part, n_parts, overlap, h->opt.tile, h->opt.block_target);
    h->info.n_colours = h->S.n_colours;
    h->info.n_parts = n_parts;
    h->info.n_blocks = (int32_t)h->S.blk_size.size();
    h->info.factor_bytes = h->S.fac_elems * storage_size(h->opt.precision);
    h->info.tile = h->S.tile;
    count_envelope(*h, row_ptr, col_idx);
    hp = h.release();
  });
  if (rc == DDG_OK) *out = reinterpret_cast<ddg_handle>(hp);
  return rc;
}

int ddg_refactor(ddg_handle hd, const double* val_dev) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && val_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    DDG_HIP(hipMemcpyAsync(h->val.p, val_dev, (size_t)h->S.nnz * sizeof(double), hipMemcpyDeviceToDevice,
                           h->stream));
    numeric_setup(*h);
  });
}

int ddg_solve(ddg_handle hd, const double* f_dev, double* u_dev, ddg_info* info) {
  Handle* h = H(hd);
  int rc = guarded([&]() {
    DDG_REQUIRE(h && f_dev && u_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    hipStream_t s = h->stream;
    hipEvent_t e0, e1;
    DDG_HIP(hipEventCreate(&e0));
    DDG_HIP(hipEventCreate(&e1));
    DDG_HIP(hipEventRecord(e0, s));
    double* x = u_dev;
    double* z = h->z.as<double>();
    const size_t sb = (size_t)h->nb * sizeof(CgState);
    const int chunk = h->opt.check_every;
    int enqueued = 0;
    if (h->ic && h->nc > 0) DDG_HIP(hipMemsetAsync(h->ic_it.p, 0, (size_t)h->nb * sizeof(int32_t), s));
    if (h->persist) {
      launch_persist(*h, f_dev, x, s);
    } else {
      launch_cg_init(*h, f_dev, x, s);
      h->cur_tag = 0;
      launch_precond(*h, h->r.as<double>(), z, -1, true, s);
      launch_cg_start(*h, s);
    }
    while (!h->persist) {
      for (int t = 0; t < chunk; ++t) {
        launch_cg_step_a(*h, x, s);
        h->cur_tag = enqueued + t + 1;  // the preconditioner of iteration enqueued + t + 1
        launch_precond(*h, h->r.as<double>(), z, -1, true, s);
        launch_cg_step_b(*h, s);
      }
      h->cur_tag = -1;
      enqueued += chunk;
      DDG_HIP(hipMemcpyAsync(h->h_state, h->cstate.p, sb, hipMemcpyDeviceToHost, s));
      DDG_HIP(hipStreamSynchronize(s));
      if (h->profiling) flush_profile(*h);
      bool all = true;
      for (int32_t b = 0; b < h->nb && all; ++b) all = h->h_state[b].done != 0;
      if (all) break;
      DDG_REQUIRE(enqueued <= h->opt.max_iter + 2 * chunk, DDG_ERR_HIP, "internal: CG loop did not stop");
    }
    launch_true_residual(*h, f_dev, x, s);
    DDG_HIP(hipEventRecord(e1, s));
    h->solved = true;
    check_err_flag(*h, "solve");
    if (h->inner) check_err_flag(*h->inner, "solve (coarse level)");
    DDG_HIP(hipMemcpyAsync(h->h_state, h->cstate.p, sb, hipMemcpyDeviceToHost, s));
    DDG_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> ic_it((size_t)h->nb, 0);
    if (h->ic && h->nc > 0) {
      DDG_HIP(hipMemcpyAsync(ic_it.data(), h->ic_it.p, ic_it.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      DDG_HIP(hipStreamSynchronize(s));
    }
    float ms = 0.f;
    DDG_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // per system, then the aggregate: the worst of every figure, first failing status
    int32_t status = DDG_OK, iters = 0;
    double rel = 0.0, trel = 0.0;
    for (int32_t b = 0; b < h->nb; ++b) {
      const CgState& st = h->h_state[b];
      ddg_info& si = h->sys_info[b];
      si = h->info;
      si.status = st.status;
      si.iters = st.iters;
      si.rel_res = st.fnorm > 0 ? std::sqrt(st.rr) / st.fnorm : 0.0;
      si.true_rel_res = st.fnorm > 0 ? std::sqrt(st.true_rr) / st.fnorm : 0.0;
      si.n_coarse = h->cblk_n[b];
      si.n_parts = h->sub_off[b + 1] - h->sub_off[b];
      si.solve_ms = st.t_done >= st.t_start ? (double)(st.t_done - st.t_start) / h->clock_khz : 0.0;
      si.coarse_iters = ic_it[b];
      if (status == DDG_OK && st.status != DDG_OK) status = st.status;
      iters = std::max(iters, st.iters);
      rel = std::max(rel, si.rel_res);
      trel = std::max(trel, si.true_rel_res);
    }
    h->info.status = status;
    h->info.iters = iters;
    h->info.rel_res = rel;
    h->info.true_rel_res = trel;
    h->info.solve_ms = ms;
    h->info.coarse_iters = ic_it.empty() ? 0 : *std::max_element(ic_it.begin(), ic_it.end());
    if (info) *info = h->info;
    if (status != DDG_OK) {
      const char* what = status == DDG_ERR_NO_CONVERGENCE ? "maximum iterations reached"
                         : status == DDG_ERR_BREAKDOWN    ? "CG breakdown (p^T q <= 0 or non-finite)"
                                                          : "non-finite right-hand side";
      throw Error{status, what};
    }
  });
  if (rc != DDG_OK && info && h) {
    info->status = rc;
  }
  return rc;
}

int ddg_solve_batched(ddg_handle hd, const double* f_dev, double* u_dev, ddg_info* infos) {
  Handle* h = H(hd);
  const int rc = ddg_solve(hd, f_dev, u_dev, nullptr);
  if (h && infos && !h->host_only && (int32_t)h->sys_info.size() == h->nb)
    for (int32_t b = 0; b < h->nb; ++b) infos[b] = h->sys_info[b];
  return rc;
}

int ddg_batch_layout(ddg_handle hd, int32_t* nb, int64_t* row_off, int32_t* sub_off) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && !h->host_only, DDG_ERR_INVALID_ARG, "null or analysis-only handle");
    if (nb) *nb = h->nb;
    if (row_off) std::copy(h->seg_off.begin(), h->seg_off.end(), row_off);
    if (sub_off) std::copy(h->sub_off.begin(), h->sub_off.end(), sub_off);
  });
}

int ddg_apply_precond(ddg_handle hd, const double* r_dev, double* z_dev) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && r_dev && z_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    launch_precond(*h, r_dev, z_dev, -1, false, h->stream);
    if (h->profiling) flush_profile(*h);
  });
}

int ddg_apply_precond_stages(ddg_handle hd, const double* r_dev, double* e_dev, int32_t stages) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && r_dev && e_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    DDG_REQUIRE(stages >= 0 && stages <= 2 * h->S.n_colours + 1, DDG_ERR_INVALID_ARG, "stage count out of range");
    launch_precond(*h, r_dev, e_dev, stages, false, h->stream);
    if (h->profiling) flush_profile(*h);
  });
}

int ddg_spmv(ddg_handle hd, const double* x_dev, double* y_dev) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && x_dev && y_dev && !h->host_only, DDG_ERR_INVALID_ARG, "null argument or analysis-only handle");
    launch_spmv(*h, x_dev, y_dev, h->stream);
    DDG_HIP(hipGetLastError());
  });
}

int ddg_cg_history(ddg_handle hd, int32_t system, double* alpha, double* beta, double* rel_res, int32_t cap,
                   int32_t* count) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && !h->host_only, DDG_ERR_INVALID_ARG, "null or analysis-only handle");
    DDG_REQUIRE(system >= 0 && system < h->nb, DDG_ERR_INVALID_ARG, "system out of range");
    DDG_REQUIRE(h->solved, DDG_ERR_INVALID_ARG, "no solve has run on this handle");
    DDG_REQUIRE(cap >= 0, DDG_ERR_INVALID_ARG, "negative capacity");
    const int64_t M = (int64_t)h->opt.max_iter + 1;
    std::vector<double> hv((size_t)(3 * M));
    DDG_HIP(hipMemcpyAsync(hv.data(), h->hist.as<double>() + (int64_t)system * 3 * M, hv.size() * sizeof(double),
                           hipMemcpyDeviceToHost, h->stream));
    DDG_HIP(hipStreamSynchronize(h->stream));
    const CgState& st = h->h_state[system];
    const int32_t it = st.iters;
    if (count) *count = it;
    const double f2 = hv[2 * M];
    for (int32_t j = 0; j < cap; ++j) {
      if (alpha && j < it) alpha[j] = hv[j];
      if (beta && j + 1 < it) beta[j] = hv[M + j];
      if (rel_res && j <= it) rel_res[j] = f2 > 0 ? std::sqrt(hv[2 * M + j] / f2) : 0.0;
    }
  });
}

int ddg_cg_report_get(ddg_handle hd, int32_t system, ddg_cg_report* out) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(out, DDG_ERR_INVALID_ARG, "null argument");
    int32_t it = 0;
    const int32_t cap = h ? h->opt.max_iter + 1 : 0;
    std::vector<double> a((size_t)std::max(cap, 1)), b((size_t)std::max(cap, 1)), r((size_t)std::max(cap, 1));
    const int rc = ddg_cg_history(hd, system, a.data(), b.data(), r.data(), cap, &it);
    if (rc != DDG_OK) throw Error{rc, ddg_last_error()};
    const double tol = h->opt.rtol;
    ddg_cg_report rep{};
    rep.iters = it;
    rep.frac_iters = std::nan("");
    for (int32_t j = 0; j <= it; ++j) {
      if (r[j] <= tol) {
        if (j == 0) {
          rep.frac_iters = 0.0;
        } else {
          const double la = std::log(r[j - 1]), lb = std::log(r[j]);
          rep.frac_iters = (j - 1) + (std::log(tol) - la) / (lb - la);
        }
        break;
      }
    }
    rep.lambda_min = rep.lambda_max = rep.kappa = std::nan("");
    rep.iter_bound = -1;
    if (it > 0) {
      std::vector<double> d((size_t)it), e((size_t)std::max(it - 1, 1));
      for (int32_t j = 0; j < it; ++j) {
        d[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
        if (j + 1 < it) e[j] = std::sqrt(b[j]) / a[j];
      }
      tridiag_extremes(d, e, rep.lambda_min, rep.lambda_max);
      rep.kappa = rep.lambda_max / rep.lambda_min;
      if (rep.kappa <= 1.0) {
        rep.iter_bound = tol >= 2.0 ? 0 : 1;
      } else {
        const double q = (std::sqrt(rep.kappa) - 1.0) / (std::sqrt(rep.kappa) + 1.0);
        rep.iter_bound = std::max(0, (int32_t)std::ceil(std::log(tol / 2.0) / std::log(q)));
      }
    }
    *out = rep;
  });
}

int ddg_get_info(ddg_handle hd, ddg_info* info) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && info, DDG_ERR_INVALID_ARG, "null argument");
    *info = h->info;
    info->sweep_groups = h->grp_used;
  });
}

int ddg_export(ddg_handle hd, int32_t what, void* host_buf, int64_t bytes, int64_t* bytes_needed) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h, DDG_ERR_INVALID_ARG, "null handle");
    const Symbolic& S = h->S;
    const void* src = nullptr;
    int64_t need = 0;
    bool device = false;
    std::vector<int32_t> blocks;
    switch (what) {
      case DDG_EXPORT_COLOURS: src = S.colour.data(); need = (int64_t)S.colour.size() * 4; break;
      case DDG_EXPORT_SET_PTR: src = S.set_ptr.data(); need = (int64_t)S.set_ptr.size() * 8; break;
      case DDG_EXPORT_SET_IDX: src = S.set_idx.data(); need = (int64_t)S.set_idx.size() * 4; break;
      case DDG_EXPORT_KCOUNTS:
        DDG_REQUIRE(!h->host_only, DDG_ERR_INVALID_ARG, "analysis-only handle");
        src = h->kcnt.data(); need = (int64_t)h->kcnt.size() * 4; break;
      case DDG_EXPORT_A0:
        DDG_REQUIRE(!h->host_only, DDG_ERR_INVALID_ARG, "analysis-only handle");
        src = h->A0.p; need = (h->nc > 0 ? h->a0_off[h->nb] : 0) * 8; device = true; break;
      case DDG_EXPORT_Q:
        DDG_REQUIRE(!h->host_only, DDG_ERR_INVALID_ARG, "analysis-only handle");
        src = h->Q.p; need = S.n * h->k * 8; device = true; break;
      case DDG_EXPORT_BLOCKS:
        for (int32_t i = 0; i < S.n_parts; ++i)
          for (int32_t b = S.sub_blk_ptr[i]; b < S.sub_blk_ptr[i + 1]; ++b) {
            blocks.push_back(i);
            blocks.push_back(S.blk_start[b]);
            blocks.push_back(S.blk_size[b]);
          }
        src = blocks.data();
        need = (int64_t)blocks.size() * 4;
        break;
      default: throw Error{DDG_ERR_INVALID_ARG, "unknown export item"};
    }
    if (bytes_needed) *bytes_needed = need;
    if (!host_buf) return;
    DDG_REQUIRE(bytes == need, DDG_ERR_INVALID_ARG, "buffer size mismatch: need " + std::to_string(need));
    if (need == 0) return;
    if (device) {
      DDG_HIP(hipMemcpyAsync(host_buf, src, need, hipMemcpyDeviceToHost, h->stream));
      DDG_HIP(hipStreamSynchronize(h->stream));
    } else {
      std::memcpy(host_buf, src, need);
    }
  });
}

int ddg_profile_enable(ddg_handle hd, int32_t on) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && !h->host_only, DDG_ERR_INVALID_ARG, "null or analysis-only handle");
    flush_profile(*h);
    h->profiling = on != 0;
  });
}

int ddg_profile_read(ddg_handle hd, double* ms, int64_t* launches, int64_t* bytes, int32_t reset) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && !h->host_only, DDG_ERR_INVALID_ARG, "null or analysis-only handle");
    flush_profile(*h);
    if (ms) *ms = h->prof_ms;
    if (launches) *launches = h->prof_launches;
    if (bytes) *bytes = h->prof_bytes;
    if (reset) {
      h->prof_ms = 0.0;
      h->prof_launches = 0;
      h->prof_bytes = 0;
      h->prof_idle_ms = 0.0;
      h->prof_idle_launches = 0;
    }
  });
}

int ddg_profile_read_idle(ddg_handle hd, double* ms, int64_t* launches) {
  return guarded([&]() {
    Handle* h = H(hd);
    DDG_REQUIRE(h && !h->host_only, DDG_ERR_INVALID_ARG, "null or analysis-only handle");
    flush_profile(*h);
    if (ms) *ms = h->prof_idle_ms;
    if (launches) *launches = h->prof_idle_launches;
  });
}

void ddg_destroy(ddg_handle hd) {
  Handle* h = H(hd);
  if (!h) return;
  if (!h->host_only) (void)hipStreamSynchronize(h->stream);
  delete h;
}

}  // extern "C"
