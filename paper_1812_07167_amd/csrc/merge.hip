// Merge-stage data movement (Sec. 2.2, Algorithm 1 step (6)) and the solve-stage
// gathers/scatters of Algorithm 2.
//
// Every box keeps its boundary in the canonical order [S, E, N, W] (each side in
// ascending coordinate).  For a merge, codeA/codeB classify each child boundary
// position as I1/I2 (exterior) or I3 (shared) with its index inside that set, and
// perm maps the parent's boundary [I1; I2] (the order Sec. 2.2 gives it) to the
// parent's canonical order.  The extract kernel reads each child R once and writes
// the blocks R33, R31, R13 (alpha), R33, R32, R23 (beta) that the merge products take.
// The parent R is written whole by the two products blockdiag(R13, R23) [Phi^a; Phi^b]
// (rows I1, then I2, every column), after which the diagonal blocks R11 and R22 are
// added from the children in place (eq. (out)), so the parent R needs no zero fill.
#include "kernels.hpp"

namespace hps {
namespace {

__global__ void fill_zero_kernel(double* p, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    p[e] = 0.0;
}

__global__ void to_f32_kernel(const double* s, float* d, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (float)s[e];
}

__global__ void to_f64_kernel(const float* s, double* d, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    d[e] = (double)s[e];
}

__global__ void fill_zero_int_kernel(int* p, long n) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    p[e] = 0;
}

template <class T>
__global__ void fill_identity_kernel(typename Cx<T>::t* p, int n, long stride, int batch) {
  const long tot = (long)n * n * batch;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const long b = e / ((long)n * n);
    const int loc = e % ((long)n * n);
    const int i = loc % n, j = loc / n;
    p[b * stride + loc] = Cx<T>::mk(i == j ? T(1) : T(0), T(0));
  }
}

// Tc: element type of the children's R; Tp: element type of the level's blocks (a
// complex128 child feeding a complex64 level is rounded here)
template <class Tc, class Tp>
__global__ void extract_kernel(MergeLevelDesc d) {
  typedef typename Cx<Tc>::t Cc;
  typedef typename Cx<Tp>::t Cp;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nn = (long)d.nbc * d.nbc;
  if (e >= nn) return;
  const int side = blockIdx.z;
  const int i = e % d.nbc, j = e / d.nbc;
  for (long q = blockIdx.y; q < d.nbox; q += gridDim.y) {
  const Cc* R = reinterpret_cast<const Cc*>(d.Rc) + (2 * q + side) * nn;
  const Cc w = R[e];
  const Cp v = Cx<Tp>::mk((Tp)w.x, (Tp)w.y);
  const Cp nv = Cx<Tp>::mk(-v.x, -v.y);
  const int n1 = d.n1, n2 = d.n2, n3 = d.n3, nbp = d.nbp;
  if (side == 0) {
    const int ci = d.codeA[i], cj = d.codeA[j];
    const int ti = ci >> 16, ki = ci & 0xffff, tj = cj >> 16, kj = cj & 0xffff;
    if (ti == 1 && tj == 1) {
      reinterpret_cast<Cp*>(d.R33a)[q * n3 * n3 + ki + (long)n3 * kj] = v;
    } else if (ti == 1 && tj == 0) {
      reinterpret_cast<Cp*>(d.R31a)[q * n3 * n1 + ki + (long)n3 * kj] = v;
      reinterpret_cast<Cp*>(d.PhiB)[q * n3 * nbp + ki + (long)n3 * d.perm[kj]] = nv;
    } else if (ti == 0 && tj == 1) {
      reinterpret_cast<Cp*>(d.R13a)[q * n1 * n3 + ki + (long)n1 * kj] = v;
    }
  } else {
    const int ci = d.codeB[i], cj = d.codeB[j];
    const int ti = ci >> 16, ki = ci & 0xffff, tj = cj >> 16, kj = cj & 0xffff;
    if (ti == 1 && tj == 1) {
      reinterpret_cast<Cp*>(d.R33b)[q * n3 * n3 + ki + (long)n3 * kj] = v;
    } else if (ti == 1 && tj == 0) {
      reinterpret_cast<Cp*>(d.T)[q * n3 * nbp + ki + (long)n3 * d.perm[n1 + kj]] = nv;
    } else if (ti == 0 && tj == 1) {
      reinterpret_cast<Cp*>(d.R23b)[q * n2 * n3 + ki + (long)n2 * kj] = v;
    }
  }
  }  // boxes
}

// Parent R += blockdiag(R11^a, R22^b) in canonical order: entry (i, j) of I1 x I1 comes
// from alpha's R at (i1a[i], i1a[j]), of I2 x I2 from beta's at (i2b[i], i2b[j]).
template <class Tc, class Tp>
__global__ void add_diag_kernel(MergeLevelDesc d) {
  typedef typename Cx<Tc>::t Cc;
  typedef typename Cx<Tp>::t Cp;
  const int side = blockIdx.z;
  const int nk = side ? d.n2 : d.n1;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)nk * nk) return;
  const int i = e % nk, j = e / nk;
  const long nn = (long)d.nbc * d.nbc;
  for (long q = blockIdx.y; q < d.nbox; q += gridDim.y) {
  const Cc* R = reinterpret_cast<const Cc*>(d.Rc) + (2 * q + side) * nn;
  const int* pos = side ? d.i2b : d.i1a;
  const int* pm = d.perm + (side ? d.n1 : 0);
  const Cc w = R[pos[i] + (long)d.nbc * pos[j]];
  Cp* P = reinterpret_cast<Cp*>(d.Rp) + q * (long)d.nbp * d.nbp + pm[i] + (long)d.nbp * pm[j];
  Cp v = *P;
  v.x += (Tp)w.x;
  v.y += (Tp)w.y;
  *P = v;
  }  // boxes
}

__global__ void leaf_h_kernel(int nleaf, int n, int nb, int nrhs, const double* prm, int nl1,
                              const double2* u, double2* h, PrmTab tab, bool use_tab) {
  const long per = (long)nb * nrhs;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < per * nleaf;
       e += (long)gridDim.x * blockDim.x) {
    const long b = e / per;
    const int loc = e % per;
    const int k = loc % nb, r = loc / nb;
    // the leaf's problem: kappa, Re eta, Im eta
    const double* pp = use_tab ? tab.p[b / nl1] : prm + 4 * (b / nl1);
    const double2 x = u[b * (long)n * nrhs + k + (long)n * r];
    h[e] = cmul(cmk(2.0 * pp[2], -2.0 * pp[1]), x);
  }
}

__global__ void up_gather_kernel(MergeLevelDesc d, int nrhs, const double2* hc, double2* h3a,
                                 double2* v, double2* ttb, double2* hp, const double2* jmp,
                                 long ldj, const int* ja, const int* jb, long jbase) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = d.n1, n2 = d.n2, n3 = d.n3, nbc = d.nbc, nbp = d.nbp;
  const int rows = n3 + n1 + n2;
  if (e >= rows * nrhs) return;
  const int k = e % rows, r = e / rows;
  for (long q = blockIdx.y; q < d.nbox; q += gridDim.y) {
  const double2* ha = hc + (2 * q) * (long)nbc * nrhs;
  const double2* hb = hc + (2 * q + 1) * (long)nbc * nrhs;
  if (k < n3) {
    double2 a = ha[d.i3a[k] + (long)nbc * r];
    double2 bb = hb[d.i3b[k] + (long)nbc * r];
    if (jmp) {
      const long qk = q * (long)n3 + k;
      a = csub(a, jmp[(long)r * ldj + jb[qk] - jbase]);    // h3a - j2
      bb = csub(bb, jmp[(long)r * ldj + ja[qk] - jbase]);  // h3b - j1
    }
    const long o = q * (long)n3 * nrhs + k + (long)n3 * r;
    h3a[o] = a;
    ttb[o] = make_double2(-a.x, -a.y);
    v[o] = make_double2(-bb.x, -bb.y);
  } else if (k < n3 + n1) {
    const int kk = k - n3;
    hp[q * (long)nbp * nrhs + d.perm[kk] + (long)nbp * r] = ha[d.i1a[kk] + (long)nbc * r];
  } else {
    const int kk = k - n3 - n1;
    hp[q * (long)nbp * nrhs + d.perm[n1 + kk] + (long)nbp * r] = hb[d.i2b[kk] + (long)nbc * r];
  }
  }  // boxes
}

__global__ void down_scatter_kernel(MergeLevelDesc d, int nrhs, const double2* tp, long ldp,
                                    double2* tc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int n1 = d.n1, n2 = d.n2, nbc = d.nbc, nbp = d.nbp;
  const int rows = n1 + n2;
  if (e >= rows * nrhs) return;
  const int k = e % rows, r = e / rows;
  for (long q = blockIdx.y; q < d.nbox; q += gridDim.y) {
  const double2* t = tp + q * (long)nbp * nrhs;
  if (k < n1) {
    tc[(2 * q) * (long)nbc * nrhs + d.i1a[k] + (long)nbc * r] = t[d.perm[k] + ldp * r];
  } else {
    const int kk = k - n1;
    tc[(2 * q + 1) * (long)nbc * nrhs + d.i2b[kk] + (long)nbc * r] = t[d.perm[n1 + kk] + ldp * r];
  }
  }  // boxes
}

}  // namespace

void fill_zero(double* p, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid1d(n)), dim3(256), 0, st, p, n);
  HPS_LAUNCH_CHECK();
}

void to_c64(const double* src, float* dst, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid1d(n)), dim3(256), 0, st, src, dst, n);
  HPS_LAUNCH_CHECK();
}

void to_c128(const float* src, double* dst, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(to_f64_kernel, dim3(grid1d(n)), dim3(256), 0, st, src, dst, n);
  HPS_LAUNCH_CHECK();
}

void fill_zero_int(int* p, long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_zero_int_kernel, dim3(grid1d(n)), dim3(256), 0, st, p, n);
  HPS_LAUNCH_CHECK();
}

void fill_identity(double* p, int n, long stride, int batch, hipStream_t st, bool c64) {
  long tot = (long)n * n * batch;
  if (tot <= 0) return;
  if (c64)
    hipLaunchKernelGGL(fill_identity_kernel<float>, dim3(grid1d(tot)), dim3(256), 0, st,
                       reinterpret_cast<float2*>(p), n, stride, batch);
  else
    hipLaunchKernelGGL(fill_identity_kernel<double>, dim3(grid1d(tot)), dim3(256), 0, st,
                       reinterpret_cast<double2*>(p), n, stride, batch);
  HPS_LAUNCH_CHECK();
}

void merge_extract(const MergeLevelDesc& d, hipStream_t st) {
  long nn = (long)d.nbc * d.nbc;
  const dim3 grid(cdiv(nn, 256), grid_y(d.nbox), 2);
  if (d.child_c64 && d.c64)
    hipLaunchKernelGGL((extract_kernel<float, float>), grid, dim3(256), 0, st, d);
  else if (d.c64)
    hipLaunchKernelGGL((extract_kernel<double, float>), grid, dim3(256), 0, st, d);
  else if (d.child_c64)
    hipLaunchKernelGGL((extract_kernel<float, double>), grid, dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL((extract_kernel<double, double>), grid, dim3(256), 0, st, d);
  HPS_LAUNCH_CHECK();
}

void merge_add_diag(const MergeLevelDesc& d, hipStream_t st) {
  const long nk = std::max(d.n1, d.n2);
  const dim3 grid(cdiv(nk * nk, 256), grid_y(d.nbox), 2);
  if (d.child_c64 && d.c64)
    hipLaunchKernelGGL((add_diag_kernel<float, float>), grid, dim3(256), 0, st, d);
  else if (d.c64)
    hipLaunchKernelGGL((add_diag_kernel<double, float>), grid, dim3(256), 0, st, d);
  else if (d.child_c64)
    hipLaunchKernelGGL((add_diag_kernel<float, double>), grid, dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL((add_diag_kernel<double, double>), grid, dim3(256), 0, st, d);
  HPS_LAUNCH_CHECK();
}

void leaf_h_from_u(int nleaf, int n, int nb, int nrhs, const double* prm, int nl1,
                   const double* u, double* h, hipStream_t st, const PrmTab* tab) {
  long tot = (long)nleaf * nb * nrhs;
  const PrmTab t = tab ? *tab : PrmTab();
  hipLaunchKernelGGL(leaf_h_kernel, dim3(grid1d(tot)), dim3(256), 0, st, nleaf, n, nb, nrhs,
                     prm, nl1, reinterpret_cast<const double2*>(u), reinterpret_cast<double2*>(h),
                     t, tab != nullptr);
  HPS_LAUNCH_CHECK();
}

void up_gather(const MergeLevelDesc& d, int nrhs, const double* hc, double* h3a, double* v,
               double* ttb, double* hp, const double* jmp, long ldj, const int* ja,
               const int* jb, long jbase, hipStream_t st) {
  long rows = (long)(d.n3 + d.n1 + d.n2) * nrhs;
  hipLaunchKernelGGL(up_gather_kernel, dim3(cdiv(rows, 256), grid_y(d.nbox)), dim3(256), 0, st, d, nrhs,
                     reinterpret_cast<const double2*>(hc), reinterpret_cast<double2*>(h3a),
                     reinterpret_cast<double2*>(v), reinterpret_cast<double2*>(ttb),
                     reinterpret_cast<double2*>(hp), reinterpret_cast<const double2*>(jmp), ldj,
                     ja, jb, jbase);
  HPS_LAUNCH_CHECK();
}

void down_scatter(const MergeLevelDesc& d, int nrhs, const double* tp, long ldp, double* tc,
                  hipStream_t st) {
  long rows = (long)(d.n1 + d.n2) * nrhs;
  hipLaunchKernelGGL(down_scatter_kernel, dim3(cdiv(rows, 256), grid_y(d.nbox)), dim3(256), 0, st, d,
                     nrhs, reinterpret_cast<const double2*>(tp), ldp,
                     reinterpret_cast<double2*>(tc));
  HPS_LAUNCH_CHECK();
}

}  // namespace hps
