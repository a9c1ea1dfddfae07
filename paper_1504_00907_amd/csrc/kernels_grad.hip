// Cell-centred harmonic-mean diffusion operator on an nx x ny x nz grid
// (x fastest), kappa = exp(theta): assembly of its CSR values and the
// per-cell coefficient gradient of a solve-based loss.  The grid is 3D when
// nz > 1, 2D when nz = 1 < ny, else 1D; ghost faces exist only along the
// grid's own axes.
//
// Face between cells L and R: a = 2 kL kR / (kL + kR), entries -a off the
// diagonal, +a on both diagonals; a boundary face with a zero-Dirichlet ghost
// adds 2 kc.  Which boundary faces have one is the ddg_bc choice: all of them
// (DDG_BC_DIRICHLET) or only those on x = 0 (DDG_BC_X0, the other faces
// carrying no flux, as in the 3D Poisson problem of Section 7).  For L(u), A u = f, the adjoint lam (A lam = dL/du) gives
//   dL/dtheta_c = -kappa_c * lam^T (dA/dkappa_c) u
//              = -kappa_c [ sum_faces 2 k_o^2/(k_c+k_o)^2 (lam_c-lam_o)(u_c-u_o)
//                           + sum_boundary_faces 2 lam_c u_c ].
#include "common.hpp"

namespace ddg {

namespace {

struct Grid {
  int nx, ny, nz;
  int bc;  // ddg_bc
};

// Boundary faces of a cell that carry a zero-Dirichlet ghost, in the order
// z-1, y-1, x-1, x+1, y+1, z+1; only the grid's own axes have faces.
__device__ inline void ghost_faces(const Grid& G, bool active[6]) {
  const bool ay = G.ny > 1 || G.nz > 1, az = G.nz > 1;  // grid dimension: 3 if nz > 1, 2 if ny > 1
  const bool all = G.bc == DDG_BC_DIRICHLET;
  active[0] = az && all;
  active[1] = ay && all;
  active[2] = true;
  active[3] = all;
  active[4] = ay && all;
  active[5] = az && all;
}

// Stored entries of all rows before cell (x, y, z) in sorted-column CSR order.
__device__ inline int64_t entries_before(const Grid& G, int x, int y, int z) {
  auto pair_cnt = [](int64_t c, int64_t m) -> int64_t {  // sum over c' < c of (c'>0)+(c'<m-1)
    if (c <= 0) return 0;
    return (c - 1) + (c < m - 1 ? c : m - 1);
  };
  const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
  const int64_t g = x + nx * (y + ny * (int64_t)z);
  int64_t cnt = g;  // diagonals
  // x neighbours
  const int64_t full_rows = y + ny * (int64_t)z;
  cnt += full_rows * 2 * (nx - 1) + pair_cnt(x, nx);
  // y neighbours
  cnt += (int64_t)z * nx * 2 * (ny - 1) + nx * pair_cnt(y, ny) + (int64_t)x * ((y > 0) + (y < ny - 1));
  // z neighbours
  cnt += nx * ny * pair_cnt(z, nz) + (y * nx + (int64_t)x) * ((z > 0) + (z < nz - 1));
  return cnt;
}

__global__ void k_assemble(Grid G, const double* __restrict__ theta, double* __restrict__ val) {
  const int64_t n = (int64_t)G.nx * G.ny * G.nz;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int x = (int)(g % G.nx), y = (int)((g / G.nx) % G.ny), z = (int)(g / ((int64_t)G.nx * G.ny));
  const double kc = exp(theta[g]);
  const int64_t sx = 1, sy = G.nx, sz = (int64_t)G.nx * G.ny;
  double off[6];
  bool has[6];
  double diag = 0.0;
  // order: z-1, y-1, x-1, x+1, y+1, z+1
  const int64_t nb[6] = {g - sz, g - sy, g - sx, g + sx, g + sy, g + sz};
  const bool in[6] = {z > 0, y > 0, x > 0, x < G.nx - 1, y < G.ny - 1, z < G.nz - 1};
  bool active[6];
  ghost_faces(G, active);
  for (int d = 0; d < 6; ++d) {
    has[d] = in[d];
    off[d] = 0.0;
    if (in[d]) {
      const double ko = exp(theta[nb[d]]);
      const double a = 2.0 * kc * ko / (kc + ko);
      off[d] = -a;
      diag += a;
    } else if (active[d]) {
      diag += 2.0 * kc;
    }
  }
  int64_t p = entries_before(G, x, y, z);
  for (int d = 0; d < 3; ++d)
    if (has[d]) val[p++] = off[d];
  val[p++] = diag;
  for (int d = 3; d < 6; ++d)
    if (has[d]) val[p++] = off[d];
}

__global__ void k_coeff_grad(Grid G, const double* __restrict__ theta, const double* __restrict__ u,
                             const double* __restrict__ lam, double* __restrict__ grad) {
  const int64_t n = (int64_t)G.nx * G.ny * G.nz;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int x = (int)(g % G.nx), y = (int)((g / G.nx) % G.ny), z = (int)(g / ((int64_t)G.nx * G.ny));
  const double kc = exp(theta[g]);
  const double uc = u[g], lc = lam[g];
  const int64_t sx = 1, sy = G.nx, sz = (int64_t)G.nx * G.ny;
  const int64_t nb[6] = {g - sz, g - sy, g - sx, g + sx, g + sy, g + sz};
  const bool in[6] = {z > 0, y > 0, x > 0, x < G.nx - 1, y < G.ny - 1, z < G.nz - 1};
  bool active[6];
  ghost_faces(G, active);
  double acc = 0.0;
  for (int d = 0; d < 6; ++d) {
    if (in[d]) {
      const double ko = exp(theta[nb[d]]);
      const double s = kc + ko;
      acc += 2.0 * ko * ko / (s * s) * (lc - lam[nb[d]]) * (uc - u[nb[d]]);
    } else if (active[d]) {
      acc += 2.0 * lc * uc;
    }
  }
  grad[g] = -kc * acc;
}

}  // namespace

}  // namespace ddg

using namespace ddg;

extern "C" int ddg_stencil_assemble(const int32_t dims[3], const double* theta_dev, int32_t bc, double* val_dev,
                                    void* stream) {
  try {
    clear_error();
    DDG_REQUIRE(dims && dims[0] > 0 && dims[1] > 0 && dims[2] > 0, DDG_ERR_INVALID_ARG, "bad grid dims");
    DDG_REQUIRE(theta_dev && val_dev, DDG_ERR_INVALID_ARG, "null pointer");
    DDG_REQUIRE(bc == DDG_BC_DIRICHLET || bc == DDG_BC_X0, DDG_ERR_INVALID_ARG, "bc must be a ddg_bc value");
    Grid G{dims[0], dims[1], dims[2], bc};
    const int64_t n = (int64_t)G.nx * G.ny * G.nz;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, G,
                       theta_dev, val_dev);
    DDG_HIP(hipGetLastError());
    return DDG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

extern "C" int ddg_stencil_coeff_grad(const int32_t dims[3], const double* theta_dev, const double* u_dev,
                                      const double* lam_dev, int32_t bc, double* grad_dev, void* stream) {
  try {
    clear_error();
    DDG_REQUIRE(dims && dims[0] > 0 && dims[1] > 0 && dims[2] > 0, DDG_ERR_INVALID_ARG, "bad grid dims");
    DDG_REQUIRE(theta_dev && u_dev && lam_dev && grad_dev, DDG_ERR_INVALID_ARG, "null pointer");
    DDG_REQUIRE(bc == DDG_BC_DIRICHLET || bc == DDG_BC_X0, DDG_ERR_INVALID_ARG, "bc must be a ddg_bc value");
    Grid G{dims[0], dims[1], dims[2], bc};
    const int64_t n = (int64_t)G.nx * G.ny * G.nz;
    hipLaunchKernelGGL(k_coeff_grad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, G,
                       theta_dev, u_dev, lam_dev, grad_dev);
    DDG_HIP(hipGetLastError());
    return DDG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
