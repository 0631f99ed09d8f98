// FP64 residual of the global collocation system that the HPS factorization eliminates
// (not in the paper: it drives the residual correction of a reduced-precision solve).
//
// Rows of leaf l (grid order), with u_l its n nodal values in the order [I_b, I_i]:
//   interior node (i, j):   s - Ahat(I_i, I) u_l,  Ahat = -Dxx - Dyy - kappa^2 c   (Sec. 2.1)
//   boundary node on dOmega: t - F u_l,             F = N + i eta on that side       (Sec. 2.1)
//   node shared with leaf l': jump - (F_l u_l + G_l' u_l'),  G = N - i eta           (Sec. 2.2)
// where N is the outward normal derivative of the leaf's own interpolant.  Matrix-free:
// the Laplacian and normal derivatives are applied with the p x p differentiation
// matrices on the leaf's full tensor grid; the four corners are never read (interior
// rows and normal rows only touch nodes off the corners).
//
// Two passes.  One workgroup per (leaf, right-hand side) puts the leaf's values into LDS
// on the full p x p grid and writes the interior rows, and the outward normal derivative
// of its own interpolant at every edge node (into the boundary rows, as scratch).  Then
// one thread per shared edge node (the leaf whose east or north side it lies on owns the
// pair) or root-boundary node combines those derivatives with the edge values into the
// impedance rows of both leaves; each boundary row is read and written by one thread.
#include "kernels.hpp"

namespace hps {
namespace {

// position of full-grid node (i, j) in a leaf vector [S, E, N, W, interior], m = p - 2;
// -1 for the corners
__device__ inline int node_pos(int i, int j, int p) {
  const int m = p - 2;
  const bool bi = (i == 0 || i == p - 1), bj = (j == 0 || j == p - 1);
  if (bi && bj) return -1;
  if (j == 0) return i - 1;                  // S
  if (i == p - 1) return m + j - 1;          // E
  if (j == p - 1) return 2 * m + i - 1;      // N
  if (i == 0) return 3 * m + j - 1;          // W
  return 4 * m + (j - 1) * m + (i - 1);      // interior
}

// Outward normal derivative, at edge node `idx` (1..p-2) of side `side` (0 S, 1 E, 2 N,
// 3 W), of the leaf whose values are read by val(i, j).
template <class V>
__device__ inline double2 normal_deriv(int side, int idx, int p, const double* Dx1,
                                       const double* Dy1, V val) {
  double2 acc = cmk(0, 0);
#pragma unroll 4
  for (int k = 0; k < p; ++k) {
    double2 x;
    double w;
    switch (side) {
      case 0: w = -Dy1[0 + p * k]; x = val(idx, k); break;             // -d/dy at y = y0
      case 1: w = Dx1[(p - 1) + p * k]; x = val(k, idx); break;        // +d/dx at x = x1
      case 2: w = Dy1[(p - 1) + p * k]; x = val(idx, k); break;        // +d/dy at y = y1
      default: w = -Dx1[0 + p * k]; x = val(k, idx); break;            // -d/dx at x = x0
    }
    // corners carry zero weight in these sums only through the zero grid entries
    acc.x += w * x.x;
    acc.y += w * x.y;
  }
  return acc;
}

template <int P>
__global__ __launch_bounds__(256) void residual_kernel(ResidualDesc d) {
  constexpr int M = P - 2, NB = 4 * M, NI = M * M, N = NB + NI;
  __shared__ double2 Ug[P * P];
  __shared__ double sD[4][P * P];
  const int tid = threadIdx.x;
  const int lg = blockIdx.x, r = blockIdx.y;   // leaf of the launch, right-hand side
  const int nl1 = d.nx * d.ny;
  const int prob = lg / nl1;                    // problem of the leaf
  const int nleaf = nl1 * d.nprob;              // leaves of the launch
  const double kappa = d.prm[4 * prob];
  for (int e = tid; e < 4 * P * P; e += 256) sD[e / (P * P)][e % (P * P)] = d.D[e];
  const double2* u = reinterpret_cast<const double2*>(d.u) + (long)r * nleaf * N;
  const double2* ul = u + (long)lg * N;
  for (int e = tid; e < P * P; e += 256) {
    const int i = e % P, j = e / P;
    const int pos = node_pos(i, j, P);
    Ug[e] = pos < 0 ? cmk(0, 0) : ul[pos];
  }
  __syncthreads();
  const double* Dx1 = sD[0];
  const double* Dy1 = sD[1];
  const double* Dxx = sD[2];
  const double* Dyy = sD[3];
  const double k2 = kappa * kappa;
  // interior rows
  for (int e = tid; e < NI; e += 256) {
    const int i = e % M + 1, j = e / M + 1;
    double2 lap = cmk(0, 0);
    // (partly unrolled: a full unroll holds every operand at once and halves occupancy)
#pragma unroll 4
    for (int k = 0; k < P; ++k) {
      const double2 a = Ug[k + P * j], b = Ug[i + P * k];
      lap.x += Dxx[i + P * k] * a.x + Dyy[j + P * k] * b.x;
      lap.y += Dxx[i + P * k] * a.y + Dyy[j + P * k] * b.y;
    }
    const double cc = k2 * d.c[(long)lg * NI + e];
    const double2 uc = Ug[i + P * j];
    const double2 Au = cmk(-lap.x - cc * uc.x, -lap.y - cc * uc.y);
    double2 b = cmk(0, 0);
    if (d.s) b = reinterpret_cast<const double2*>(d.s)[(long)r * nleaf * NI + (long)lg * NI + e];
    reinterpret_cast<double2*>(d.rs)[r * d.rs_rhs + lg * d.rs_leaf + e] = csub(b, Au);
  }
  // boundary rows: the leaf's own outward normal derivative N u_l, combined below
  double2* rb = reinterpret_cast<double2*>(d.rb) + r * d.rb_rhs + lg * d.rb_leaf;
  for (int e = tid; e < NB; e += 256) {
    auto own = [&](int i, int j) { return Ug[i + P * j]; };
    rb[e] = normal_deriv(e / M, e % M + 1, P, Dx1, Dy1, own);
  }
}

// Impedance rows from the normal derivatives the leaf pass left in rb: entry e of leaf l
// on side `side`.  A root-boundary node gives t - F u_l (F = N + i eta); a node shared
// with leaf l' (its entry e') gives jump - (F_l u_l + G_l' u_l') (G = N - i eta) for l
// and the mirror image for l'.  Threads of west and south entries with a neighbour do
// nothing: the neighbour's east or north thread writes both rows.
__global__ __launch_bounds__(256) void residual_edge_kernel(ResidualDesc d, int M) {
  const int NB = 4 * M;
  const int nl1 = d.nx * d.ny;
  const long nleaf = (long)nl1 * d.nprob;
  const long tot = (long)d.nrhs * nleaf * NB;
  const int nt = 2 * (d.nx + d.ny) * M;
  for (long g = (long)blockIdx.x * 256 + threadIdx.x; g < tot; g += (long)gridDim.x * 256) {
    const int e = (int)(g % NB);
    const long lg = (g / NB) % nleaf;
    const int r = (int)(g / (NB * nleaf));
    const int prob = (int)(lg / nl1), l = (int)(lg % nl1);
    const int ix = l % d.nx, iy = l / d.nx;
    const int side = e / M, q = e % M;
    int root = -1;
    switch (side) {
      case 0: if (iy == 0) root = ix * M + q; break;
      case 1: if (ix == d.nx - 1) root = d.nx * M + iy * M + q; break;
      case 2: if (iy == d.ny - 1) root = (d.nx + d.ny) * M + ix * M + q; break;
      default: if (ix == 0) root = (2 * d.nx + d.ny) * M + iy * M + q; break;
    }
    if (root < 0 && (side == 0 || side == 3)) continue;  // written by the neighbour
    const double eta_re = d.prm[4 * prob + 1], eta_im = d.prm[4 * prob + 2];
    // F v = N v + i eta v and G v = N v - i eta v at one node
    auto Fv = [&](double2 nd, double2 v) {
      return cmk(nd.x - eta_im * v.x - eta_re * v.y, nd.y + eta_re * v.x - eta_im * v.y);
    };
    auto Gv = [&](double2 nd, double2 v) {
      return cmk(nd.x + eta_im * v.x + eta_re * v.y, nd.y - eta_re * v.x + eta_im * v.y);
    };
    const double2* u = reinterpret_cast<const double2*>(d.u) + (long)r * nleaf * (NB + M * M);
    double2* rb = reinterpret_cast<double2*>(d.rb) + r * d.rb_rhs;
    const double2 ndl = rb[lg * d.rb_leaf + e];
    const double2 ul = u[lg * (NB + M * M) + e];
    if (root >= 0) {
      const long trow = ((long)prob * d.nrhs + r) * nt;  // t, rt: [problem][rhs][nt]
      double2 tv = cmk(0, 0);
      if (d.t) tv = reinterpret_cast<const double2*>(d.t)[trow + root];
      const double2 res = csub(tv, Fv(ndl, ul));
      if (d.rt) {
        reinterpret_cast<double2*>(d.rt)[trow + root] = res;
        rb[lg * d.rb_leaf + e] = cmk(0, 0);
      } else {
        rb[lg * d.rb_leaf + e] = res;
      }
      continue;
    }
    // east side: the neighbour's west entry q; north side: the neighbour's south entry q
    const long ln = (long)prob * nl1 + (side == 1 ? l + 1 : l + d.nx);
    const int en = (side == 1 ? 3 : 0) * M + q;
    const double2 ndn = rb[ln * d.rb_leaf + en];
    const double2 un = u[ln * (NB + M * M) + en];
    double2 jl = cmk(0, 0), jn = cmk(0, 0);
    if (d.jmp) {
      const double2* jp = reinterpret_cast<const double2*>(d.jmp) + (long)r * nleaf * NB;
      jl = jp[lg * NB + e];
      jn = jp[ln * NB + en];
    }
    rb[lg * d.rb_leaf + e] = csub(jl, cadd(Fv(ndl, ul), Gv(ndn, un)));
    rb[ln * d.rb_leaf + en] = csub(jn, cadd(Fv(ndn, un), Gv(ndl, ul)));
  }
}

__global__ void axpy_kernel(long n, const double2* x, double2* y) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    y[e] = cadd(y[e], x[e]);
}

// partial sums of |x|^2 and |y|^2 per block of one column (fixed order); columns beyond
// the grid's y extent are taken in turn
__global__ __launch_bounds__(256) void norms_kernel(long len, int ncol, const double2* x,
                                                    const double2* y, double* part) {
  __shared__ double sx[256], sy[256];
  for (long r = blockIdx.y; r < ncol; r += gridDim.y) {
  const long base = r * len;
  double ax = 0, ay = 0;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < len; e += (long)gridDim.x * 256) {
    const double2 a = x[base + e], b = y[base + e];
    ax += a.x * a.x + a.y * a.y;
    ay += b.x * b.x + b.y * b.y;
  }
  __syncthreads();  // the previous column's sums have been read
  sx[threadIdx.x] = ax;
  sy[threadIdx.x] = ay;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sx[threadIdx.x] += sx[threadIdx.x + w];
      sy[threadIdx.x] += sy[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (r * gridDim.x + blockIdx.x)] = sx[0];
    part[2 * (r * gridDim.x + blockIdx.x) + 1] = sy[0];
  }
  }  // columns
}

}  // namespace

void residual(const ResidualDesc& d, int nrhs, hipStream_t st) {
  if (nrhs <= 0) return;
  if (nrhs > 65535) throw Error(1, "residual: too many right-hand sides");
  if (nrhs != d.nrhs) throw Error(1, "residual: right-hand side count differs from the layout");
  const dim3 grid(d.nx * d.ny * d.nprob, nrhs);
  switch (d.p) {
#define HPS_RES_CASE(PP) \
  case PP: hipLaunchKernelGGL(residual_kernel<PP>, grid, dim3(256), 0, st, d); break;
    HPS_RES_CASE(4) HPS_RES_CASE(5) HPS_RES_CASE(6) HPS_RES_CASE(7) HPS_RES_CASE(8)
    HPS_RES_CASE(9) HPS_RES_CASE(10) HPS_RES_CASE(11) HPS_RES_CASE(12) HPS_RES_CASE(13)
    HPS_RES_CASE(14) HPS_RES_CASE(15) HPS_RES_CASE(16)
#undef HPS_RES_CASE
    default: throw Error(1, "residual: unsupported p");
  }
  HPS_LAUNCH_CHECK();
  const long tot = (long)nrhs * d.nx * d.ny * d.nprob * 4 * (d.p - 2);
  hipLaunchKernelGGL(residual_edge_kernel, dim3(grid1d(tot)), dim3(256), 0, st, d, d.p - 2);
  HPS_LAUNCH_CHECK();
}

void axpy(long n, const double* x, double* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(axpy_kernel, dim3(grid1d(n)), dim3(256), 0, st, n,
                     reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y));
  HPS_LAUNCH_CHECK();
}

int norms_blocks() { return 64; }

void norms_partial(long len, int nrhs, const double* x, const double* y, double* part,
                   hipStream_t st) {
  if (len <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(norms_kernel, dim3(norms_blocks(), grid_y(nrhs)), dim3(256), 0, st, len,
                     nrhs, reinterpret_cast<const double2*>(x),
                     reinterpret_cast<const double2*>(y), part);
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
