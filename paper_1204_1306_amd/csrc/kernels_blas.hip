// BLAS-1 on batches of spinor fields and deterministic two-pass reductions
// (fixed grid, fixed summation order, FP64 accumulation for every storage).
#include "kernels.h"

namespace psms {

// A storage unit seen as N consecutive complex numbers of one component plane.
template <Prec P> struct Unit;
template <> struct Unit<P_F64> {
  using unit = double2;
  using T = double;
  static constexpr int N = 1, NC = 12;
  __device__ static void ld(const unit& u, cx<T> (&c)[N]) { c[0] = {u.x, u.y}; }
  __device__ static void st(unit& u, const cx<T> (&c)[N]) { u = make_double2(c[0].re, c[0].im); }
};
template <> struct Unit<P_F32> {
  using unit = float4;
  using T = float;
  static constexpr int N = 2, NC = 6;
  __device__ static void ld(const unit& u, cx<T> (&c)[N]) { c[0] = {u.x, u.y}; c[1] = {u.z, u.w}; }
  __device__ static void st(unit& u, const cx<T> (&c)[N]) { u = make_float4(c[0].re, c[0].im, c[1].re, c[1].im); }
};
template <> struct Unit<P_BF16> {
  using unit = uint4;
  using T = float;
  static constexpr int N = 4, NC = 3;
  __device__ static void ld(const unit& u, cx<T> (&c)[N]) {
    uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = {bf16_to_f32(w[j] & 0xffffu), bf16_to_f32(w[j] >> 16)};
  }
  __device__ static void st(unit& u, const cx<T> (&c)[N]) {
    uint32_t w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = uint32_t(f32_to_bf16(c[j].re)) | (uint32_t(f32_to_bf16(c[j].im)) << 16);
    u = make_uint4(w[0], w[1], w[2], w[3]);
  }
};

#define DISPATCH_PREC(prec, KERNEL, ...)                                     \
  do {                                                                       \
    if ((prec) == P_F64) KERNEL<P_F64>(__VA_ARGS__);                         \
    else if ((prec) == P_F32) KERNEL<P_F32>(__VA_ARGS__);                    \
    else KERNEL<P_BF16>(__VA_ARGS__);                                        \
  } while (0)

static inline int nrhs_of(const FieldBatch& f) { return f.nprop * f.nrhs; }

// ----------------------------------------------------------------- axpby
template <Prec P>
__global__ void k_axpby(const double2* __restrict__ a, const typename Unit<P>::unit* __restrict__ x, const double2* __restrict__ b,
                        typename Unit<P>::unit* __restrict__ y, size_t n, double sgn) {
  using U = Unit<P>;
  using T = typename U::T;
  const int r = blockIdx.y;
  cx<double> ar = a ? cx<double>{sgn * a[r].x, sgn * a[r].y} : cx<double>{0, 0};
  cx<double> br = b ? cx<double>{b[r].x, b[r].y} : cx<double>{1, 0};
  const cx<T> A = {T(ar.re), T(ar.im)}, B = {T(br.re), T(br.im)};
  const size_t off = size_t(r) * n;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> xv[U::N], yv[U::N];
    U::ld(y[off + i], yv);
    if (a) U::ld(x[off + i], xv);
#pragma unroll
    for (int j = 0; j < U::N; ++j) yv[j] = (a ? cmul(A, xv[j]) : cx<T>{0, 0}) + cmul(B, yv[j]);
    U::st(y[off + i], yv);
  }
}

static dim3 grid1(size_t n, int nrhs) {
  size_t g = (n + 255) / 256;
  if (g > 2048) g = 2048;
  return dim3(unsigned(g), nrhs);
}

template <Prec P> static void axpby_go(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const double2* b,
                                       const FieldBatch& y, int sgn) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_axpby<P>, grid1(n, nrhs_of(y)), dim3(256), 0, st, a, (const typename Unit<P>::unit*)x.p, b,
                     (typename Unit<P>::unit*)y.p, n, double(sgn));
}
void launch_axpby(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const double2* b, const FieldBatch& y,
                  int coef_sign) {
  DISPATCH_PREC(y.prec, axpby_go, st, g, a, x, b, y, coef_sign);
}

// ----------------------------------------------------------------- zero
__global__ void k_zero(uint4* __restrict__ y, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    y[i] = make_uint4(0, 0, 0, 0);
}
void launch_zero(hipStream_t st, const FieldBatch& y, int Vh) {
  size_t n = units_per_field(y.prec, Vh) * nrhs_of(y);
  hipLaunchKernelGGL(k_zero, grid1(n, 1), dim3(256), 0, st, (uint4*)y.p, n);
}

__global__ void k_zero_parity(uint4* __restrict__ y, size_t half, int parity) {
  uint4* q = y + (size_t(blockIdx.y) * 2 + parity) * half;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < half; i += size_t(gridDim.x) * blockDim.x)
    q[i] = make_uint4(0, 0, 0, 0);
}
void launch_zero_parity(hipStream_t st, const FieldBatch& y, int Vh, int parity) {
  size_t half = units_per_field(y.prec, Vh) / 2;  // every storage unit is 16 bytes
  hipLaunchKernelGGL(k_zero_parity, grid1(half, nrhs_of(y)), dim3(256), 0, st, (uint4*)y.p, half, parity);
}

// ----------------------------------------------------------------- copy / convert (site level)
template <class SX, class SY, class T>
__global__ void k_copy(Geo g, const typename SX::unit* __restrict__ x, typename SY::unit* __restrict__ y, const double* __restrict__ s) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  int p = t / g.Vh, i = t - p * g.Vh;
  int r = blockIdx.y;
  Spinor<T> v;
  SX::load(x + (size_t(r) * 2 + p) * SX::NC * g.Vh, g.Vh, i, v);
  if (s) {
    T f = T(s[r]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) v.v[a][c] = scale(f, v.v[a][c]);
  }
  SY::store(y + (size_t(r) * 2 + p) * SY::NC * g.Vh, g.Vh, i, v);
}

template <class SX, class SY, class T> static void copy_go(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const double* s) {
  dim3 grid((2 * g.Vh + 255) / 256, nrhs_of(y));
  hipLaunchKernelGGL((k_copy<SX, SY, T>), grid, dim3(256), 0, st, g, (const typename SX::unit*)x.p, (typename SY::unit*)y.p, s);
}
void launch_copy(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const double* s) {
  if (x.prec == P_F64 && y.prec == P_F64) copy_go<StF64, StF64, double>(st, g, x, y, s);
  else if (x.prec == P_F64 && y.prec == P_F32) copy_go<StF64, StF32, double>(st, g, x, y, s);
  else if (x.prec == P_F64 && y.prec == P_BF16) copy_go<StF64, StBF16, double>(st, g, x, y, s);
  else if (x.prec == P_F32 && y.prec == P_F64) copy_go<StF32, StF64, double>(st, g, x, y, s);
  else if (x.prec == P_BF16 && y.prec == P_F64) copy_go<StBF16, StF64, double>(st, g, x, y, s);
  else if (x.prec == P_F32 && y.prec == P_F32) copy_go<StF32, StF32, float>(st, g, x, y, s);
  else if (x.prec == P_BF16 && y.prec == P_BF16) copy_go<StBF16, StBF16, float>(st, g, x, y, s);
  else if (x.prec == P_F32 && y.prec == P_BF16) copy_go<StF32, StBF16, float>(st, g, x, y, s);
  else copy_go<StBF16, StF32, float>(st, g, x, y, s);
}

// ----------------------------------------------------------------- keep one colour
template <Prec P>
__global__ void k_keep_colour(Geo g, typename Unit<P>::unit* __restrict__ y, int keep) {
  using U = Unit<P>;
  size_t n = size_t(2) * U::NC * g.Vh;
  size_t off = size_t(blockIdx.y) * n;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    int s = int(i % g.Vh);
    int col = (s / g.Vbh) >= g.nblk_c ? 1 : 0;
    if (col != keep) {
      cx<typename U::T> z[U::N];
#pragma unroll
      for (int j = 0; j < U::N; ++j) z[j] = {0, 0};
      U::st(y[off + i], z);
    }
  }
}
template <Prec P> static void keep_go(hipStream_t st, const Geo& g, const FieldBatch& y, int keep) {
  hipLaunchKernelGGL(k_keep_colour<P>, grid1(units_per_field(P, g.Vh), nrhs_of(y)), dim3(256), 0, st, g,
                     (typename Unit<P>::unit*)y.p, keep);
}
void launch_keep_colour(hipStream_t st, const Geo& g, const FieldBatch& y, int keep_colour) {
  DISPATCH_PREC(y.prec, keep_go, st, g, y, keep_colour);
}

// ----------------------------------------------------------------- interpolation
// out[i] = wx x[i] + wy y[i] for i < n: intermediate link fields, entry by entry
__global__ void k_lerp(const double* __restrict__ x, const double* __restrict__ y, double wx, double wy,
                       double* __restrict__ out, size_t n) {
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
    out[i] = wx * x[i] + wy * y[i];
}
void launch_lerp(hipStream_t st, const double* x, const double* y, double wx, double wy, double* out, size_t n) {
  if (n == 0) return;
  const size_t g = (n + 255) / 256;
  const unsigned nwg = unsigned(g < 65536 ? g : 65536);
  hipLaunchKernelGGL(k_lerp, dim3(nwg), dim3(256), 0, st, x, y, wx, wy, out, n);
}

// ----------------------------------------------------------------- linear combination
// y += sign * sum_j c[r][j] X_j
template <Prec P>
__global__ void k_lincomb(const typename Unit<P>::unit* __restrict__ basis, size_t vstride, int m, const double2* __restrict__ c,
                          int cstride, typename Unit<P>::unit* __restrict__ y, size_t n, double sgn) {
  using U = Unit<P>;
  using T = typename U::T;
  const int r = blockIdx.y;
  const size_t off = size_t(r) * n;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> yv[U::N];
    cx<double> acc[U::N];
    U::ld(y[off + i], yv);
#pragma unroll
    for (int k = 0; k < U::N; ++k) acc[k] = {double(yv[k].re), double(yv[k].im)};
    for (int j = 0; j < m; ++j) {
      cx<double> cj = {sgn * c[r * cstride + j].x, sgn * c[r * cstride + j].y};
      cx<T> xv[U::N];
      U::ld(basis[j * vstride + off + i], xv);
#pragma unroll
      for (int k = 0; k < U::N; ++k) acc[k] = acc[k] + cmul(cj, cx<double>{double(xv[k].re), double(xv[k].im)});
    }
#pragma unroll
    for (int k = 0; k < U::N; ++k) yv[k] = {T(acc[k].re), T(acc[k].im)};
    U::st(y[off + i], yv);
  }
}
template <Prec P> static void lincomb_go(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c,
                                         int cstride, const FieldBatch& y, int sign) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_lincomb<P>, grid1(n, nrhs_of(y)), dim3(256), 0, st, (const typename Unit<P>::unit*)basis.p, vstride, m, c,
                     cstride, (typename Unit<P>::unit*)y.p, n, double(sign));
}
void launch_lincomb(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c, int cstride,
                    const FieldBatch& y, int sign) {
  if (m <= 0) return;
  DISPATCH_PREC(y.prec, lincomb_go, st, g, basis, vstride, m, c, cstride, y, sign);
}

// ----------------------------------------------------------------- reductions
__device__ __forceinline__ double block_sum(double v, double* sm) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += sm[k];  // every thread sums in the same order
  return t;
}

template <Prec P>
__global__ void k_norm2_p1(const typename Unit<P>::unit* __restrict__ x, size_t n, double* __restrict__ partial) {
  using U = Unit<P>;
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * n;
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<typename U::T> v[U::N];
    U::ld(x[off + i], v);
#pragma unroll
    for (int k = 0; k < U::N; ++k) acc += double(v[k].re) * double(v[k].re) + double(v[k].im) * double(v[k].im);
  }
  double t = block_sum(acc, sm);
  if (threadIdx.x == 0) partial[size_t(r) * gridDim.x + blockIdx.x] = t;
}

// out[q] = sum_w partial[q * nwg + w] for q < nq (double entries, stride 'width' doubles per entry)
__global__ void k_reduce_final(const double* __restrict__ partial, int nwg, int width, double* __restrict__ out) {
  __shared__ double sm[16];
  const int q = blockIdx.x;
  for (int c = 0; c < width; ++c) {
    double acc = 0.0;
    for (int w = threadIdx.x; w < nwg; w += blockDim.x) acc += partial[(size_t(q) * nwg + w) * width + c];
    double t = block_sum(acc, sm);
    if (threadIdx.x == 0) out[size_t(q) * width + c] = t;
  }
}

// The last pass of reduce_multidot with the projection step of flexible GCR: entry
// q = r * k + j is (W_j, w_k)_r, summed exactly as k_reduce_final sums it; then
// a[r*m + j] = entry / nw[r*m + j] (0 when nw is 0) and T[(r*m + j)*m + k] = a.
__global__ void k_reduce_final_proj(const double* __restrict__ partial, int nwg, GcrStep gs) {
  __shared__ double sm[16];
  const int q = blockIdx.x;
  double v[2];
  for (int c = 0; c < 2; ++c) {
    double acc = 0.0;
    for (int w = threadIdx.x; w < nwg; w += blockDim.x) acc += partial[(size_t(q) * nwg + w) * 2 + c];
    v[c] = block_sum(acc, sm);
  }
  if (threadIdx.x == 0) {
    const int r = q / gs.k, j = q - r * gs.k;
    const double n = gs.nw[r * gs.m + j];
    const double2 e = n > 0 ? make_double2(v[0] / n, v[1] / n) : make_double2(0, 0);
    gs.a[r * gs.m + j] = e;
    gs.T[(size_t(r) * gs.m + j) * gs.m + gs.k] = e;
  }
}

// The last pass of reduce_norm_dot with the step length of flexible GCR: from
// {|w_k|^2, (w_k, r)} of right-hand side r (summed as k_reduce_final sums them),
// nw[r*m + k] = |w_k|^2, alpha[k*nrhs + r] = (w_k, r) / |w_k|^2 for active right-hand
// sides with a nonzero norm (else 0) and neg_alpha[r] = -alpha.
__global__ void k_reduce_final_alpha(const double* __restrict__ partial, int nwg, GcrStep gs) {
  __shared__ double sm[16];
  const int r = blockIdx.x;
  double v[3];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int w = threadIdx.x; w < nwg; w += blockDim.x) acc += partial[(size_t(r) * nwg + w) * 3 + c];
    v[c] = block_sum(acc, sm);
  }
  if (threadIdx.x == 0) {
    const double n = v[0];
    gs.nw[r * gs.m + gs.k] = n;
    const double2 e = (gs.active[r] && n > 0) ? make_double2(v[1] / n, v[2] / n) : make_double2(0, 0);
    gs.alpha[gs.k * gs.nrhs + r] = e;
    gs.neg_alpha[r] = make_double2(-e.x, -e.y);
  }
}

template <Prec P> static void norm2_go(hipStream_t st, const Geo& g, const FieldBatch& x, const Reducer& R, double* out) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_norm2_p1<P>, dim3(R.nwg, nrhs_of(x)), dim3(256), 0, st, (const typename Unit<P>::unit*)x.p, n, R.partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(nrhs_of(x)), dim3(256), 0, st, R.partial, R.nwg, 1, out);
}
void reduce_norm2(hipStream_t st, const Geo& g, const FieldBatch& x, const Reducer& R, double* out) {
  DISPATCH_PREC(x.prec, norm2_go, st, g, x, R, out);
}

// (X_j, y) for j in [j0, j0 + K), conj on X. partial layout [(r*m + j)*nwg + w][2]
template <Prec P, int K>
__global__ void k_multidot_p1(const typename Unit<P>::unit* __restrict__ basis, size_t vstride, int j0, int m,
                              const typename Unit<P>::unit* __restrict__ y, size_t n, double* __restrict__ partial) {
  using U = Unit<P>;
  using T = typename U::T;
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * n;
  const int kk = min(K, m - j0);
  double are[K], aim[K];
#pragma unroll
  for (int k = 0; k < K; ++k) are[k] = aim[k] = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> yv[U::N];
    U::ld(y[off + i], yv);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < kk) {
        cx<T> xv[U::N];
        U::ld(basis[(j0 + k) * vstride + off + i], xv);
#pragma unroll
        for (int e = 0; e < U::N; ++e) {
          are[k] += double(xv[e].re) * double(yv[e].re) + double(xv[e].im) * double(yv[e].im);
          aim[k] += double(xv[e].re) * double(yv[e].im) - double(xv[e].im) * double(yv[e].re);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (k < kk) {
      double tr = block_sum(are[k], sm);
      double ti = block_sum(aim[k], sm);
      if (threadIdx.x == 0) {
        size_t q = (size_t(r) * m + j0 + k) * gridDim.x + blockIdx.x;
        partial[2 * q] = tr;
        partial[2 * q + 1] = ti;
      }
    }
  }
}

template <Prec P> static void multidot_go(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const FieldBatch& y,
                                          const Reducer& R, double2* out, const GcrStep* gs) {
  size_t n = units_per_field(P, g.Vh);
  for (int j0 = 0; j0 < m; j0 += 16)
    hipLaunchKernelGGL((k_multidot_p1<P, 16>), dim3(R.nwg, nrhs_of(y)), dim3(256), 0, st, (const typename Unit<P>::unit*)basis.p,
                       vstride, j0, m, (const typename Unit<P>::unit*)y.p, n, R.partial);
  if (gs) hipLaunchKernelGGL(k_reduce_final_proj, dim3(nrhs_of(y) * m), dim3(256), 0, st, R.partial, R.nwg, *gs);
  else hipLaunchKernelGGL(k_reduce_final, dim3(nrhs_of(y) * m), dim3(256), 0, st, R.partial, R.nwg, 2, (double*)out);
}
void reduce_multidot(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const FieldBatch& y,
                     const Reducer& R, double2* out, const GcrStep* gs) {
  if (m <= 0) return;
  DISPATCH_PREC(y.prec, multidot_go, st, g, basis, vstride, m, y, R, out, gs);
}

// |x|^2 and (x, y) (conj on x) in one pass; partial [(r * nwg + w) * 3 + {|x|^2, Re, Im}]
template <Prec P>
__global__ void k_norm_dot_p1(const typename Unit<P>::unit* __restrict__ x, const typename Unit<P>::unit* __restrict__ y,
                              size_t n, double* __restrict__ partial) {
  using U = Unit<P>;
  using T = typename U::T;
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * n;
  double xx = 0.0, re = 0.0, im = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> xv[U::N], yv[U::N];
    U::ld(x[off + i], xv);
    U::ld(y[off + i], yv);
#pragma unroll
    for (int e = 0; e < U::N; ++e) {
      const double xr = xv[e].re, xi = xv[e].im, yr = yv[e].re, yi = yv[e].im;
      xx += xr * xr + xi * xi;
      re += xr * yr + xi * yi;
      im += xr * yi - xi * yr;
    }
  }
  const double t0 = block_sum(xx, sm), t1 = block_sum(re, sm), t2 = block_sum(im, sm);
  if (threadIdx.x == 0) {
    const size_t q = size_t(r) * gridDim.x + blockIdx.x;
    partial[3 * q] = t0;
    partial[3 * q + 1] = t1;
    partial[3 * q + 2] = t2;
  }
}
// The orthogonalisation of flexible GCR with the pass that follows it: y -= sum_j
// c[r][j] X_j (as k_lincomb with sign -1), then the partial sums of |y|^2 and (y, z)
// (conj on y) over the stored y, with the same work split and layout as k_norm_dot_p1,
// so that the sums equal those of the two passes bit for bit.
template <Prec P>
__global__ void k_lincomb_norm_dot(const typename Unit<P>::unit* __restrict__ basis, size_t vstride, int m,
                                   const double2* __restrict__ c, int cstride, typename Unit<P>::unit* __restrict__ y,
                                   const typename Unit<P>::unit* __restrict__ z, size_t n, double* __restrict__ partial) {
  using U = Unit<P>;
  using T = typename U::T;
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const size_t off = size_t(r) * n;
  double xx = 0.0, re = 0.0, im = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> yv[U::N], zv[U::N];
    cx<double> acc[U::N];
    U::ld(y[off + i], yv);
    U::ld(z[off + i], zv);
#pragma unroll
    for (int k = 0; k < U::N; ++k) acc[k] = {double(yv[k].re), double(yv[k].im)};
    for (int j = 0; j < m; ++j) {
      cx<double> cj = {-c[r * cstride + j].x, -c[r * cstride + j].y};
      cx<T> xv[U::N];
      U::ld(basis[j * vstride + off + i], xv);
#pragma unroll
      for (int k = 0; k < U::N; ++k) acc[k] = acc[k] + cmul(cj, cx<double>{double(xv[k].re), double(xv[k].im)});
    }
#pragma unroll
    for (int k = 0; k < U::N; ++k) yv[k] = {T(acc[k].re), T(acc[k].im)};
    typename U::unit u;
    U::st(u, yv);
    y[off + i] = u;
    U::ld(u, yv);  // the stored (rounded) values enter the sums
#pragma unroll
    for (int e = 0; e < U::N; ++e) {
      const double xr = yv[e].re, xi = yv[e].im, yr = zv[e].re, yi = zv[e].im;
      xx += xr * xr + xi * xi;
      re += xr * yr + xi * yi;
      im += xr * yi - xi * yr;
    }
  }
  const double t0 = block_sum(xx, sm), t1 = block_sum(re, sm), t2 = block_sum(im, sm);
  if (threadIdx.x == 0) {
    const size_t q = size_t(r) * gridDim.x + blockIdx.x;
    partial[3 * q] = t0;
    partial[3 * q + 1] = t1;
    partial[3 * q + 2] = t2;
  }
}
template <Prec P> static void lincomb_norm_dot_go(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m,
                                                  const double2* c, int cstride, const FieldBatch& y, const FieldBatch& z,
                                                  const Reducer& R, const GcrStep& gs) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_lincomb_norm_dot<P>, dim3(R.nwg, nrhs_of(y)), dim3(256), 0, st, (const typename Unit<P>::unit*)basis.p,
                     vstride, m, c, cstride, (typename Unit<P>::unit*)y.p, (const typename Unit<P>::unit*)z.p, n, R.partial);
  hipLaunchKernelGGL(k_reduce_final_alpha, dim3(nrhs_of(y)), dim3(256), 0, st, R.partial, R.nwg, gs);
}
void lincomb_norm_dot(hipStream_t st, const Geo& g, const FieldBatch& basis, size_t vstride, int m, const double2* c, int cstride,
                      const FieldBatch& y, const FieldBatch& z, const Reducer& R, const GcrStep& gs) {
  DISPATCH_PREC(y.prec, lincomb_norm_dot_go, st, g, basis, vstride, m, c, cstride, y, z, R, gs);
}

template <Prec P> static void norm_dot_go(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                                          double* out3, const GcrStep* gs) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_norm_dot_p1<P>, dim3(R.nwg, nrhs_of(x)), dim3(256), 0, st, (const typename Unit<P>::unit*)x.p,
                     (const typename Unit<P>::unit*)y.p, n, R.partial);
  if (gs) hipLaunchKernelGGL(k_reduce_final_alpha, dim3(nrhs_of(x)), dim3(256), 0, st, R.partial, R.nwg, *gs);
  else hipLaunchKernelGGL(k_reduce_final, dim3(nrhs_of(x)), dim3(256), 0, st, R.partial, R.nwg, 3, out3);
}
void reduce_norm_dot(hipStream_t st, const Geo& g, const FieldBatch& x, const FieldBatch& y, const Reducer& R, double* out3,
                     const GcrStep* gs) {
  DISPATCH_PREC(x.prec, norm_dot_go, st, g, x, y, R, out3, gs);
}

// y += a[r] * x and the partial sums of |y|^2 (new y) in one pass
template <Prec P>
__global__ void k_axpy_norm_p1(const double2* __restrict__ a, const typename Unit<P>::unit* __restrict__ x,
                               typename Unit<P>::unit* __restrict__ y, size_t n, double* __restrict__ partial) {
  using U = Unit<P>;
  using T = typename U::T;
  __shared__ double sm[16];
  const int r = blockIdx.y;
  const cx<T> A = {T(a[r].x), T(a[r].y)};
  const size_t off = size_t(r) * n;
  double acc = 0.0;
  for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
    cx<T> xv[U::N], yv[U::N];
    U::ld(x[off + i], xv);
    U::ld(y[off + i], yv);
#pragma unroll
    for (int e = 0; e < U::N; ++e) yv[e] = yv[e] + cmul(A, xv[e]);
    typename U::unit u;
    U::st(u, yv);
    y[off + i] = u;
    cx<T> zv[U::N];  // the stored (rounded) values enter the norm
    U::ld(u, zv);
#pragma unroll
    for (int e = 0; e < U::N; ++e) acc += double(zv[e].re) * double(zv[e].re) + double(zv[e].im) * double(zv[e].im);
  }
  const double t = block_sum(acc, sm);
  if (threadIdx.x == 0) partial[size_t(r) * gridDim.x + blockIdx.x] = t;
}
template <Prec P> static void axpy_norm_go(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y,
                                           const Reducer& R, double* out) {
  size_t n = units_per_field(P, g.Vh);
  hipLaunchKernelGGL(k_axpy_norm_p1<P>, dim3(R.nwg, nrhs_of(y)), dim3(256), 0, st, a, (const typename Unit<P>::unit*)x.p,
                     (typename Unit<P>::unit*)y.p, n, R.partial);
  hipLaunchKernelGGL(k_reduce_final, dim3(nrhs_of(y)), dim3(256), 0, st, R.partial, R.nwg, 1, out);
}
void axpy_norm2(hipStream_t st, const Geo& g, const double2* a, const FieldBatch& x, const FieldBatch& y, const Reducer& R,
                double* out) {
  DISPATCH_PREC(y.prec, axpy_norm_go, st, g, a, x, y, R, out);
}


// out[r * nblk + blk] = |x|^2 over the sites of block blk (both parities) of FP64 field r:
// one workgroup per (block, field), a fixed-order tree in LDS (deterministic).
__global__ void __launch_bounds__(256) k_block_norm2(Geo g, const double2* __restrict__ x, double* __restrict__ out) {
  __shared__ double sm[256];
  const int blk = blockIdx.x, r = blockIdx.y, t = threadIdx.x;
  const size_t Vh = g.Vh;
  const double2* f = x + size_t(r) * 24 * Vh + size_t(blk) * g.Vbh;
  const int per = 12 * g.Vbh;  // units of one parity of a block
  double acc = 0.0;
  for (int e = t; e < 2 * per; e += 256) {
    const int p = e / per, rem = e - p * per, k = rem / g.Vbh, i = rem - k * g.Vbh;
    const double2 v = f[(size_t(p) * 12 + k) * Vh + i];
    acc += v.x * v.x + v.y * v.y;
  }
  sm[t] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sm[t] += sm[t + o];
    __syncthreads();
  }
  if (t == 0) out[size_t(r) * g.nblk + blk] = sm[0];
}

void launch_block_norm2(hipStream_t st, const Geo& g, const FieldBatch& x, double* out) {
  hipLaunchKernelGGL(k_block_norm2, dim3(g.nblk, x.nprop * x.nrhs), dim3(256), 0, st, g, (const double2*)x.p, out);
}
}  // namespace psms
