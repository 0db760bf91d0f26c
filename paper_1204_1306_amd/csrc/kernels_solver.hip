// Small per-right-hand-side scalar kernels of the flexible GCR and mixed-storage
// site-level BLAS (a low-precision Krylov basis against an FP32 residual).
#include "kernels.h"

namespace psms {

// alpha[k*nrhs + r] = d[r] / nw[r*m + k] for active right-hand sides, else 0
__global__ void k_gcr_alpha(const double2* __restrict__ d, const double* __restrict__ nw, int k, int m, int nrhs,
                            const int* __restrict__ active, double2* __restrict__ alpha, double2* __restrict__ neg_alpha) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double n = nw[r * m + k];
  double2 v = (active[r] && n > 0) ? make_double2(d[r].x / n, d[r].y / n) : make_double2(0, 0);
  alpha[k * nrhs + r] = v;
  neg_alpha[r] = make_double2(-v.x, -v.y);
}

// beta solves T beta = alpha (unit upper triangular), beta laid out [r*m + j]
__global__ void k_gcr_backsub(const double2* __restrict__ T, const double2* __restrict__ alpha, int n, int m, int nrhs,
                              double2* __restrict__ beta) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  for (int k = n - 1; k >= 0; --k) {
    cx<double> acc = {alpha[k * nrhs + r].x, alpha[k * nrhs + r].y};
    for (int j = k + 1; j < n; ++j) {
      double2 t = T[(size_t(r) * m + k) * m + j];
      acc = acc - cmul(cx<double>{t.x, t.y}, cx<double>{beta[r * m + j].x, beta[r * m + j].y});
    }
    beta[r * m + k] = make_double2(acc.re, acc.im);
  }
}

void gcr_alpha(hipStream_t st, const double2* d, const double* nw, int k, int m, int nrhs, const int* active, double2* alpha,
               double2* neg_alpha) {
  hipLaunchKernelGGL(k_gcr_alpha, dim3((nrhs + 255) / 256), dim3(256), 0, st, d, nw, k, m, nrhs, active, alpha, neg_alpha);
}
void gcr_backsub(hipStream_t st, const double2* T, const double2* alpha, int n, int m, int nrhs, double2* beta) {
  hipLaunchKernelGGL(k_gcr_backsub, dim3((nrhs + 63) / 64), dim3(64), 0, st, T, alpha, n, m, nrhs, beta);
}

// norm of each column of nw (|w_k|^2) copied from a per-rhs array
__global__ void k_scatter_col(const double* __restrict__ src, int k, int m, int nrhs, double* __restrict__ dst) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < nrhs) dst[r * m + k] = src[r];
}
void scatter_col(hipStream_t st, const double* src, int k, int m, int nrhs, double* dst) {
  hipLaunchKernelGGL(k_scatter_col, dim3((nrhs + 255) / 256), dim3(256), 0, st, src, k, m, nrhs, dst);
}

// s[r] = f(v[r]) helpers for defect correction: inv[r] = 1/sqrt(v) (0 if inactive), sq[r] = sqrt(v)
__global__ void k_scales(const double* __restrict__ v, const int* __restrict__ active, int nrhs, double* __restrict__ inv,
                         double2* __restrict__ sq) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = sqrt(v[r]);
  bool on = active[r] && s > 0;
  inv[r] = on ? 1.0 / s : 0.0;
  sq[r] = make_double2(on ? s : 0.0, 0.0);
}
void defect_scales(hipStream_t st, const double* v, const int* active, int nrhs, double* inv, double2* sq) {
  hipLaunchKernelGGL(k_scales, dim3((nrhs + 255) / 256), dim3(256), 0, st, v, active, nrhs, inv, sq);
}

// ---------------------------------------------------------------- mixed-storage site-level ops
// y += sign * a[r] * x   (x and y of different storage)
template <class SX, class SY, class T>
__global__ void k_axpy_site(Geo g, const double2* __restrict__ a, const typename SX::unit* __restrict__ x,
                            typename SY::unit* __restrict__ y, double sgn) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  int p = t / g.Vh, i = t - p * g.Vh, r = blockIdx.y;
  cx<T> A = {T(sgn * a[r].x), T(sgn * a[r].y)};
  Spinor<T> xv, yv;
  SX::load(x + (size_t(r) * 2 + p) * SX::NC * g.Vh, g.Vh, i, xv);
  SY::load(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, yv);
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) yv.v[q][c] = yv.v[q][c] + cmul(A, xv.v[q][c]);
  SY::store(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, yv);
}

void launch_axpy_mixed(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, int sgn) {
  dim3 grid((2 * g.Vh + 255) / 256, y.nprop * y.nrhs);
  if (x.prec == P_BF16 && y.prec == P_F32)
    hipLaunchKernelGGL((k_axpy_site<StBF16, StF32, float>), grid, dim3(256), 0, st, g, a, (const uint4*)x.p, (float4*)y.p, double(sgn));
  else if (x.prec == P_F32 && y.prec == P_BF16)
    hipLaunchKernelGGL((k_axpy_site<StF32, StBF16, float>), grid, dim3(256), 0, st, g, a, (const float4*)x.p, (uint4*)y.p, double(sgn));
  else if (x.prec == P_F32 && y.prec == P_F64)
    hipLaunchKernelGGL((k_axpy_site<StF32, StF64, double>), grid, dim3(256), 0, st, g, a, (const float4*)x.p, (double2*)y.p, double(sgn));
  else if (x.prec == P_BF16 && y.prec == P_F64)
    hipLaunchKernelGGL((k_axpy_site<StBF16, StF64, double>), grid, dim3(256), 0, st, g, a, (const uint4*)x.p, (double2*)y.p, double(sgn));
}

// y += sign * sum_{j < m} c[r * cstride + j] X_j, X_j = x + j * vstride (units of SX): the
// solution update of a restart cycle from a basis in another storage, one pass over y
template <class SX, class SY, class T>
__global__ void k_lincomb_site(Geo g, const double2* __restrict__ c, int cstride, int m,
                               const typename SX::unit* __restrict__ x, size_t vstride, typename SY::unit* __restrict__ y,
                               double sgn) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  int p = t / g.Vh, i = t - p * g.Vh, r = blockIdx.y;
  Spinor<T> yv;
  SY::load(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, yv);
  for (int j = 0; j < m; ++j) {
    const double2 cj = c[size_t(r) * cstride + j];
    const cx<T> A = {T(sgn * cj.x), T(sgn * cj.y)};
    Spinor<T> xv;
    SX::load(x + size_t(j) * vstride + (size_t(r) * 2 + p) * SX::NC * g.Vh, g.Vh, i, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) yv.v[q][cc] = yv.v[q][cc] + cmul(A, xv.v[q][cc]);
  }
  SY::store(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, yv);
}

bool launch_lincomb_mixed(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c,
                          int cstride, const FieldBatch& y, int sgn) {
  if (m <= 0) return true;
  dim3 grid((2 * g.Vh + 255) / 256, y.nprop * y.nrhs);
  if (basis.prec == P_BF16 && y.prec == P_F32)
    hipLaunchKernelGGL((k_lincomb_site<StBF16, StF32, float>), grid, dim3(256), 0, st, g, c, cstride, m,
                       (const uint4*)basis.p, vstride, (float4*)y.p, double(sgn));
  else if (basis.prec == P_F32 && y.prec == P_F64)
    hipLaunchKernelGGL((k_lincomb_site<StF32, StF64, double>), grid, dim3(256), 0, st, g, c, cstride, m,
                       (const float4*)basis.p, vstride, (double2*)y.p, double(sgn));
  else if (basis.prec == P_BF16 && y.prec == P_F64)
    hipLaunchKernelGGL((k_lincomb_site<StBF16, StF64, double>), grid, dim3(256), 0, st, g, c, cstride, m,
                       (const uint4*)basis.p, vstride, (double2*)y.p, double(sgn));
  else
    return false;
  return true;
}

// partial (x, y) per workgroup at site level; final pass shared with the unit-level reducer
template <class SX, class SY>
__global__ void k_dot_site(Geo g, const typename SX::unit* __restrict__ x, const typename SY::unit* __restrict__ y,
                           double* __restrict__ partial) {
  __shared__ double sm[16];
  int r = blockIdx.y;
  double are = 0, aim = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * g.Vh; t += gridDim.x * blockDim.x) {
    int p = t / g.Vh, i = t - p * g.Vh;
    Spinor<float> xv, yv;
    SX::load(x + (size_t(r) * 2 + p) * SX::NC * g.Vh, g.Vh, i, xv);
    SY::load(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, yv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double xr = xv.v[q][c].re, xi = xv.v[q][c].im, yr = yv.v[q][c].re, yi = yv.v[q][c].im;
        are += xr * yr + xi * yi;
        aim += xr * yi - xi * yr;
      }
  }
  are = wave_sum(are);
  aim = wave_sum(aim);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) { sm[2 * w] = are; sm[2 * w + 1] = aim; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tr = 0, ti = 0;
    for (int k = 0; k < nw; ++k) { tr += sm[2 * k]; ti += sm[2 * k + 1]; }
    size_t q = size_t(r) * gridDim.x + blockIdx.x;
    partial[2 * q] = tr;
    partial[2 * q + 1] = ti;
  }
}

__global__ void k_reduce_pairs(const double* __restrict__ partial, int nwg, double* __restrict__ out) {
  int r = blockIdx.x;
  if (threadIdx.x == 0) {
    double tr = 0, ti = 0;
    for (int w = 0; w < nwg; ++w) { tr += partial[2 * (size_t(r) * nwg + w)]; ti += partial[2 * (size_t(r) * nwg + w) + 1]; }
    out[2 * r] = tr;
    out[2 * r + 1] = ti;
  }
}

void reduce_dot_mixed(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R, double2* out) {
  dim3 grid(R.nwg, y.nprop * y.nrhs);
  if (x.prec == P_BF16 && y.prec == P_F32)
    hipLaunchKernelGGL((k_dot_site<StBF16, StF32>), grid, dim3(256), 0, st, g, (const uint4*)x.p, (const float4*)y.p, R.partial);
  else
    hipLaunchKernelGGL((k_dot_site<StF32, StBF16>), grid, dim3(256), 0, st, g, (const float4*)x.p, (const uint4*)y.p, R.partial);
  hipLaunchKernelGGL(k_reduce_pairs, dim3(y.nprop * y.nrhs), dim3(64), 0, st, R.partial, R.nwg, (double*)out);
}


// |x|^2 and (x, y) in one site-level pass for a BF16 x and an FP32 y;
// partial [(r * nwg + w) * 3 + {|x|^2, Re, Im}]
__global__ void k_norm_dot_bf16_f32(Geo g, const uint4* __restrict__ x, const float4* __restrict__ y,
                                    double* __restrict__ partial) {
  __shared__ double sm[3][16];
  const int r = blockIdx.y;
  double xx = 0, re = 0, im = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * g.Vh; t += gridDim.x * blockDim.x) {
    const int p = t / g.Vh, i = t - p * g.Vh;
    Spinor<float> xv, yv;
    StBF16::load(x + (size_t(r) * 2 + p) * StBF16::NC * g.Vh, g.Vh, i, xv);
    StF32::load(y + (size_t(r) * 2 + p) * StF32::NC * g.Vh, g.Vh, i, yv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double xr = xv.v[q][c].re, xi = xv.v[q][c].im, yr = yv.v[q][c].re, yi = yv.v[q][c].im;
        xx += xr * xr + xi * xi;
        re += xr * yr + xi * yi;
        im += xr * yi - xi * yr;
      }
  }
  xx = wave_sum(xx);
  re = wave_sum(re);
  im = wave_sum(im);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    sm[0][w] = xx;
    sm[1][w] = re;
    sm[2][w] = im;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0;
    for (int k = 0; k < nw; ++k) {
      a += sm[0][k];
      b += sm[1][k];
      c += sm[2][k];
    }
    const size_t q = size_t(r) * gridDim.x + blockIdx.x;
    partial[3 * q] = a;
    partial[3 * q + 1] = b;
    partial[3 * q + 2] = c;
  }
}

// y += a[r] x (BF16 x, FP32 y) and the partial sums of |y|^2 in one site-level pass
__global__ void k_axpy_norm_bf16_f32(Geo g, const double2* __restrict__ a, const uint4* __restrict__ x,
                                     float4* __restrict__ y, double* __restrict__ partial) {
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const cx<float> A = {float(a[r].x), float(a[r].y)};
  double acc = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < 2 * g.Vh; t += gridDim.x * blockDim.x) {
    const int p = t / g.Vh, i = t - p * g.Vh;
    Spinor<float> xv, yv;
    StBF16::load(x + (size_t(r) * 2 + p) * StBF16::NC * g.Vh, g.Vh, i, xv);
    float4* yp = y + (size_t(r) * 2 + p) * StF32::NC * g.Vh;
    StF32::load(yp, g.Vh, i, yv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        yv.v[q][c] = yv.v[q][c] + cmul(A, xv.v[q][c]);
        acc += double(yv.v[q][c].re) * yv.v[q][c].re + double(yv.v[q][c].im) * yv.v[q][c].im;
      }
    StF32::store(yp, g.Vh, i, yv);  // FP32 storage holds these float values exactly
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) sm[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int k = 0; k < nw; ++k) s += sm[k];
    partial[size_t(r) * gridDim.x + blockIdx.x] = s;
  }
}

// out[r * width + c] = sum_w partial[(r * nwg + w) * width + c], in order
__global__ void k_reduce_width(const double* __restrict__ partial, int nwg, int width, double* __restrict__ out) {
  const int r = blockIdx.x;
  if (threadIdx.x < width) {
    double s = 0;
    for (int w = 0; w < nwg; ++w) s += partial[(size_t(r) * nwg + w) * width + threadIdx.x];
    out[size_t(r) * width + threadIdx.x] = s;
  }
}

bool fused_mixed_ok(const FieldBatch& x, const FieldBatch& y) { return x.prec == P_BF16 && y.prec == P_F32; }

// k_reduce_width (width 3) with the step length of flexible GCR: from the three sums
// {|w_k|^2, (w_k, r)} of right-hand side r, nw[r*m + k] = |w_k|^2, alpha[k*nrhs + r] =
// (w_k, r) / |w_k|^2 for active right-hand sides with a nonzero norm (else 0) and
// neg_alpha[r] = -alpha
__global__ void k_reduce_width_alpha(const double* __restrict__ partial, int nwg, GcrStep gs) {
  __shared__ double v[3];
  const int r = blockIdx.x;
  if (threadIdx.x < 3) {
    double s = 0;
    for (int w = 0; w < nwg; ++w) s += partial[(size_t(r) * nwg + w) * 3 + threadIdx.x];
    v[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double n = v[0];
    gs.nw[r * gs.m + gs.k] = n;
    const double2 e = (gs.active[r] && n > 0) ? make_double2(v[1] / n, v[2] / n) : make_double2(0, 0);
    gs.alpha[gs.k * gs.nrhs + r] = e;
    gs.neg_alpha[r] = make_double2(-e.x, -e.y);
  }
}

void reduce_norm_dot_mixed(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                           double* out3, const GcrStep* gs) {
  dim3 grid(R.nwg, y.nprop * y.nrhs);
  hipLaunchKernelGGL(k_norm_dot_bf16_f32, grid, dim3(256), 0, st, g, (const uint4*)x.p, (const float4*)y.p, R.partial);
  if (gs) hipLaunchKernelGGL(k_reduce_width_alpha, dim3(y.nprop * y.nrhs), dim3(64), 0, st, R.partial, R.nwg, *gs);
  else hipLaunchKernelGGL(k_reduce_width, dim3(y.nprop * y.nrhs), dim3(64), 0, st, R.partial, R.nwg, 3, out3);
}

void axpy_norm2_mixed(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                      double* out) {
  dim3 grid(R.nwg, y.nprop * y.nrhs);
  hipLaunchKernelGGL(k_axpy_norm_bf16_f32, grid, dim3(256), 0, st, g, a, (const uint4*)x.p, (float4*)y.p, R.partial);
  hipLaunchKernelGGL(k_reduce_width, dim3(y.nprop * y.nrhs), dim3(64), 0, st, R.partial, R.nwg, 1, out);
}

}  // namespace psms
