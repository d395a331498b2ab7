// gfx950 kernel of the smoothed vertex update of the shape step.
//
// The paper's shape optimisation (Sec. 5.2) moves the vertices along the
// loss gradient filtered by (I + lambda L)^{-2}, L the Laplacian of the mesh
// graph, which spreads each vertex's gradient over its neighbourhood and
// lets large steps keep the mesh regular.  Here L = D - A is the
// combinatorial graph Laplacian (D the vertex degrees, A the adjacency of the
// mesh edges) and the two solves with I + lambda L (symmetric positive
// definite for lambda >= 0) are done by conjugate gradients with the Jacobi
// preconditioner diag(I + lambda L) = 1 + lambda deg.
//
// One workgroup solves the three systems of a gradient (its x, y and z
// components, vertex-major [n_v][3] like the gradient itself) at once: the
// mesh is small (10^3 - 10^5 vertices), the iteration count is what costs,
// and a single workgroup synchronises with barriers instead of kernel
// launches.  Dot products are accumulated in float64 and reduced in a fixed
// order, so results are bitwise reproducible.  The loop ends once every
// component's residual is below tol times its right-hand side, or after
// max_iter iterations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <utility>

#include "dm_internal.h"

namespace dm {
namespace {

constexpr int CG_T = 1024;
constexpr int ADJ_W = LAP_TABLE_W;
constexpr int CG_W = CG_T / 64;

struct CgLds {
  double part[CG_W][6];
  double tot[6];
};

// One DPP lane move of a double (both halves with the same control); lanes
// the move does not write read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int64_t b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

// Sum over the 64 lanes in a fixed order (within quads, half rows, rows, then
// row pairs); the total ends in lane 63.
__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_d<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xF>(v);   // row_half_mirror
  v += dpp_d<0x140, 0xF>(v);   // row_mirror
  v += dpp_d<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_d<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Sum of v[0..N-1] over the workgroup (fixed order), returned to every thread.
template <int N>
__device__ void block_sum(double (&v)[N], CgLds& L) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const double s = wave_sum_d(v[c]);
    if (lane == 63) L.part[w][c] = s;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
    for (int i = 0; i < CG_W; ++i) s += L.part[i][threadIdx.x];
    L.tot[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < N; ++c) v[c] = L.tot[c];
  __syncthreads();
}

// (I + lam L) x = b by Jacobi-preconditioned CG; b, x, r, p, q are [nv][3].
// b is read only before x is first written, so x may be the array b.
// Returns the iterations used and writes the worst relative residual of the
// three components to *res.
// q_i = (I + lam L) p at vertex i: from the fixed-width neighbour table
// (TABLE, every degree <= ADJ_W, unused slots -1: the neighbour loads do not
// depend on each other) or from the CSR lists.
template <bool TABLE>
__device__ __forceinline__ void lap_row(int i, const int32_t* __restrict__ off, const int32_t* __restrict__ nbr,
                                        const int32_t* __restrict__ tab, const float* __restrict__ p, float s[3],
                                        int& deg) {
  s[0] = s[1] = s[2] = 0.0f;
  if (TABLE) {
    const int4 a = reinterpret_cast<const int4*>(tab)[2 * i], b = reinterpret_cast<const int4*>(tab)[2 * i + 1];
    const int nb[ADJ_W] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    deg = 0;
#pragma unroll
    for (int k = 0; k < ADJ_W; ++k) {
      if (nb[k] >= 0) {
        ++deg;
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += p[3 * nb[k] + c];
      }
    }
  } else {
    const int o0 = off[i], o1 = off[i + 1];
    deg = o1 - o0;
    for (int o = o0; o < o1; ++o) {
      const int j = nbr[o];
#pragma unroll
      for (int c = 0; c < 3; ++c) s[c] += p[3 * j + c];
    }
  }
}

// Chebyshev iteration for (I + lam L) x = b on meshes the resident CG does
// not hold: the spectrum of I + lam L lies in [1, 1 + lam mu] (L = D - A has
// the eigenvalue 0 on constant vectors, and its largest eigenvalue is at most
// mu = the largest d_i + d_j over the mesh edges, the bound of Anderson and
// Morley), so with theta and delta the centre and half-width of that interval
// and sigma = theta / delta the three-term recurrence
//   x_{k+1} = x_k + d_k,   r_{k+1} = r_k - A d_k,
//   rho_{k+1} = 1 / (2 sigma - rho_k),
//   d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1} / delta) r_{k+1},
// started from x_0 = 0, r_0 = b, rho_0 = 1 / sigma, d_0 = b / theta, reduces
// every column's residual by at least 2 rho^k after k steps, rho =
// (sqrt(kappa) - 1) / (sqrt(kappa) + 1), kappa = 1 + lam mu.  It needs no inner
// products: each step is one launch over the vertices (the neighbour sum of
// d from the previous step is the only exchange), with its two coefficients
// from the host.

// x = 0, r = b, d = b / theta.  x may be the array b (b is read first).
__global__ void k_cheb_init(int nv, const float* b, float* x, float* __restrict__ r, float* __restrict__ d,
                            float inv_theta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nv) return;
  const float bi = b[i];
  r[i] = bi;
  d[i] = bi * inv_theta;
  x[i] = 0.0f;
}

// One step: with q = (I + lam L) d at vertex i, x += d, r -= q and, unless it
// is the last step, d_next = c1 d + c2 r.  d is read at the neighbours, so the
// next direction goes to another array.
template <bool TABLE>
__global__ void k_cheb_step(int nv, const int32_t* __restrict__ off, const int32_t* __restrict__ nbr,
                            const int32_t* __restrict__ tab, float lam, const float* __restrict__ d,
                            float* __restrict__ x, float* __restrict__ r, float* __restrict__ d_next, float c1,
                            float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  float s[3];
  int deg;
  lap_row<TABLE>(i, off, nbr, tab, d, s, deg);
  const float dg = fmaf(lam, (float)deg, 1.0f);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float di = d[3 * i + c];
    const float q = fmaf(dg, di, -lam * s[c]);
    x[3 * i + c] += di;
    const float ri = r[3 * i + c] - q;
    r[3 * i + c] = ri;
    if (d_next != nullptr) d_next[3 * i + c] = fmaf(c1, di, c2 * ri);
  }
}

// info[0], info[1] = steps, worst relative residual of the three columns
// (||r|| / ||b|| in float64, summed in a fixed order by one workgroup).
__global__ void __launch_bounds__(CG_T) k_cheb_residual(int nv, const float* __restrict__ r,
                                                        const float* __restrict__ b, float steps,
                                                        float* __restrict__ info) {
  __shared__ CgLds L;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nv; i += CG_T)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] += (double)r[3 * i + c] * r[3 * i + c];
      v[3 + c] += (double)b[3 * i + c] * b[3 * i + c];
    }
  block_sum<6>(v, L);
  if (threadIdx.x == 0) {
    double worst = 0.0;
    for (int c = 0; c < 3; ++c)
      if (v[3 + c] > 0.0) worst = fmax(worst, sqrt(v[c] / v[3 + c]));
    info[0] = steps;
    info[1] = (float)worst;
  }
}

// Resident variant for meshes of at most CG_T * CG_VPT_MAX vertices whose degrees
// fit the neighbour table: thread t owns vertices t + k CG_T (k < VPT) and
// keeps their x, r, 1/d and neighbour lists in registers; only p, which the
// Laplacian product reads at the neighbours, lives in LDS.  An iteration
// then makes no global-memory round trip.  Same algorithm, same stopping
// rule and float64 reductions as cg_solve.
constexpr int CG_VPT_MAX = 3;   // 4 would exceed the 128 VGPRs of a 1024-lane workgroup

template <int VPT>
__device__ int cg_solve_res(int nv, const int (&nb)[VPT][ADJ_W], const float (&dinv)[VPT], const float (&d)[VPT],
                            float lam, float (&x)[VPT][3], const float (&b)[VPT][3], float (*p_lds)[3], int max_iter,
                            float tol, float* res, CgLds& L) {
  float r[VPT][3];
  double bz[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int i = threadIdx.x + k * CG_T;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      r[k][c] = b[k][c];
      x[k][c] = 0.0f;
      if (i < nv) {
        p_lds[i][c] = b[k][c] * dinv[k];
        bz[c] += (double)b[k][c] * b[k][c];
        bz[3 + c] += (double)b[k][c] * (b[k][c] * dinv[k]);
      }
    }
  }
  block_sum<6>(bz, L);   // its barriers also publish p
  const double bb[3] = {bz[0], bz[1], bz[2]};
  double rz[3] = {bz[3], bz[4], bz[5]}, rr[3] = {bz[0], bz[1], bz[2]};
  const double tol2 = (double)tol * tol;
  int it = 0;
  for (; it < max_iter; ++it) {
    if (rr[0] <= tol2 * bb[0] && rr[1] <= tol2 * bb[1] && rr[2] <= tol2 * bb[2]) break;
    float q[VPT][3], pk[VPT][3];
    double pq[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * CG_T;
      float s3[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < ADJ_W; ++j)
        if (nb[k][j] >= 0) {
#pragma unroll
          for (int c = 0; c < 3; ++c) s3[c] += p_lds[nb[k][j]][c];
        }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        pk[k][c] = i < nv ? p_lds[i][c] : 0.0f;
        q[k][c] = fmaf(d[k], pk[k][c], -lam * s3[c]);
        pq[c] += (double)pk[k][c] * q[k][c];
      }
    }
    block_sum<3>(pq, L);
    float alpha[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) alpha[c] = pq[c] > 0.0 ? (float)(rz[c] / pq[c]) : 0.0f;
    double rn[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < VPT; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[k][c] = fmaf(alpha[c], pk[k][c], x[k][c]);
        r[k][c] = fmaf(-alpha[c], q[k][c], r[k][c]);
        rn[c] += (double)r[k][c] * r[k][c];
        rn[3 + c] += (double)r[k][c] * (r[k][c] * dinv[k]);
      }
    block_sum<6>(rn, L);   // all reads of p for this iteration are done
    float beta[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      beta[c] = rz[c] > 0.0 ? (float)(rn[3 + c] / rz[c]) : 0.0f;
      rz[c] = rn[3 + c];
      rr[c] = rn[c];
    }
#pragma unroll
    for (int k = 0; k < VPT; ++k) {
      const int i = threadIdx.x + k * CG_T;
      if (i < nv)
#pragma unroll
        for (int c = 0; c < 3; ++c) p_lds[i][c] = fmaf(beta[c], pk[k][c], r[k][c] * dinv[k]);
    }
    __syncthreads();
  }
  double worst = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (bb[c] > 0.0) worst = fmax(worst, sqrt(rr[c] / bb[c]));
  *res = (float)worst;
  return it;
}

template <int VPT>
__global__ void __launch_bounds__(CG_T) k_laplace_smooth_res(int nv, const int32_t* __restrict__ tab, float lam,
                                                              const float* g, float* out, int max_iter, float tol,
                                                              float* __restrict__ info) {
  __shared__ CgLds L;
  __shared__ float p_lds[CG_T * VPT][3];
  int nb[VPT][ADJ_W];
  float dinv[VPT], d[VPT], b[VPT][3], x[VPT][3];
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int i = threadIdx.x + k * CG_T;
    int deg = 0;
#pragma unroll
    for (int j = 0; j < ADJ_W; ++j) {
      nb[k][j] = i < nv ? tab[(size_t)i * ADJ_W + j] : -1;
      deg += nb[k][j] >= 0 ? 1 : 0;
    }
    d[k] = fmaf(lam, (float)deg, 1.0f);
    dinv[k] = 1.0f / d[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) b[k][c] = i < nv ? g[3 * i + c] : 0.0f;
  }
  float res1 = 0.0f, res2 = 0.0f;
  const int it1 = cg_solve_res<VPT>(nv, nb, dinv, d, lam, x, b, p_lds, max_iter, tol, &res1, L);
#pragma unroll
  for (int k = 0; k < VPT; ++k)
#pragma unroll
    for (int c = 0; c < 3; ++c) b[k][c] = x[k][c];
  __syncthreads();
  const int it2 = cg_solve_res<VPT>(nv, nb, dinv, d, lam, x, b, p_lds, max_iter, tol, &res2, L);
#pragma unroll
  for (int k = 0; k < VPT; ++k) {
    const int i = threadIdx.x + k * CG_T;
    if (i < nv)
#pragma unroll
      for (int c = 0; c < 3; ++c) out[3 * i + c] = x[k][c];
  }
  if (info != nullptr && threadIdx.x == 0) {
    info[0] = (float)it1;
    info[1] = res1;
    info[2] = (float)it2;
    info[3] = res2;
  }
}

}  // namespace

size_t laplace_smooth_workspace(int nv) { return sizeof(float) * 13 * (size_t)nv; }

int chebyshev_steps(float lam, int mu, float tol, int max_iter) {
  const double kappa = 1.0 + (double)lam * (double)mu;
  if (!(kappa > 1.0)) return 0;
  const double sk = std::sqrt(kappa), rho = (sk - 1.0) / (sk + 1.0);
  const double k = std::ceil(std::log(2.0 / (double)tol) / -std::log(rho));
  return (int)std::max(1.0, std::min((double)max_iter, k));
}

namespace {

// One Chebyshev solve (see k_cheb_step): b, x [nv][3]; r, d0, d1 work arrays.
hipError_t cheb_solve(int nv, const int32_t* adj_off, const int32_t* adj_nbr, const int32_t* adj_tab, float lam,
                      int mu, int steps, const float* b, float* x, float* r, float* d0, float* d1, float* info,
                      hipStream_t s) {
  const double lo = 1.0, hi = 1.0 + (double)lam * (double)mu;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  const unsigned b3 = (unsigned)((3 * (int64_t)nv + 255) / 256), b1 = (unsigned)((nv + 255) / 256);
  hipLaunchKernelGGL(k_cheb_init, dim3(b3), dim3(256), 0, s, nv, b, x, r, d0, (float)(1.0 / theta));
  double rho = 1.0 / sigma;
  float* d = d0;
  float* dn = d1;
  for (int k = 0; k < steps; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    const bool last = k + 1 == steps;
    const float c1 = (float)(rho1 * rho), c2 = (float)(2.0 * rho1 / delta);
    if (adj_tab != nullptr)
      hipLaunchKernelGGL(k_cheb_step<true>, dim3(b1), dim3(256), 0, s, nv, adj_off, adj_nbr, adj_tab, lam, d, x, r,
                         last ? nullptr : dn, c1, c2);
    else
      hipLaunchKernelGGL(k_cheb_step<false>, dim3(b1), dim3(256), 0, s, nv, adj_off, adj_nbr, adj_tab, lam, d, x, r,
                         last ? nullptr : dn, c1, c2);
    rho = rho1;
    std::swap(d, dn);
  }
  if (info != nullptr) hipLaunchKernelGGL(k_cheb_residual, dim3(1), dim3(CG_T), 0, s, nv, r, b, (float)steps, info);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_laplace_smooth(int nv, const int32_t* adj_off, const int32_t* adj_nbr, const int32_t* adj_tab,
                                 int mu, float lam, const float* g, float* out, float* ws, int max_iter, float tol,
                                 float* info, hipStream_t s) {
  if (adj_tab != nullptr && nv <= CG_T * CG_VPT_MAX) {
    const int vpt = (nv + CG_T - 1) / CG_T;
    if (vpt <= 1)
      hipLaunchKernelGGL(k_laplace_smooth_res<1>, dim3(1), dim3(CG_T), 0, s, nv, adj_tab, lam, g, out, max_iter, tol,
                         info);
    else if (vpt == 2)
      hipLaunchKernelGGL(k_laplace_smooth_res<2>, dim3(1), dim3(CG_T), 0, s, nv, adj_tab, lam, g, out, max_iter, tol,
                         info);
    else
      hipLaunchKernelGGL(k_laplace_smooth_res<3>, dim3(1), dim3(CG_T), 0, s, nv, adj_tab, lam, g, out, max_iter, tol,
                         info);
    return hipGetLastError();
  }
  const int steps = chebyshev_steps(lam, mu, tol, max_iter);
  const size_t n3 = (size_t)3 * nv;
  float* y = ws;
  float* r = ws + n3;
  float* d0 = ws + 2 * n3;
  float* d1 = ws + 3 * n3;
  if (steps == 0) {   // I + lam L = I (lam = 0 or no edges): out = g
    if (out != g) {
      const hipError_t e = hipMemcpyAsync(out, g, n3 * sizeof(float), hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return e;
    }
    if (info != nullptr) {
      hipLaunchKernelGGL(k_cheb_residual, dim3(1), dim3(CG_T), 0, s, 0, y, g, 0.0f, info);
      hipLaunchKernelGGL(k_cheb_residual, dim3(1), dim3(CG_T), 0, s, 0, y, g, 0.0f, info + 2);
    }
    return hipGetLastError();
  }
  const hipError_t e = cheb_solve(nv, adj_off, adj_nbr, adj_tab, lam, mu, steps, g, y, r, d0, d1, info, s);
  if (e != hipSuccess) return e;
  return cheb_solve(nv, adj_off, adj_nbr, adj_tab, lam, mu, steps, y, out, r, d0, d1,
                    info != nullptr ? info + 2 : nullptr, s);
}

}  // namespace dm
