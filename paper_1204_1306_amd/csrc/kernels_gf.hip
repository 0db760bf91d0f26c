// Relative gauge fixing of a field pair (Sec. 4.2, eqs. relgf, choiceg; App. B, eqs.
// GF:fminendform, ming, GF:Delta, GF:theta), FP64, on links in the boundary layout
// [V][4][3][3] complex (lexicographic sites, x0 slowest).
//
// With g1 = g2^-1 = g the link term of eq. relgf is Re Tr{1 - U^+ G(x)^+ U' G(x+mu)} with
// G = g^2: a one-sided fixing of U' to U by G (the Landau-like form of App. B), minimised
// by steepest descent on the current field U'_G = G(x)^+ U'(x,mu) G(x+mu):
//   Delta(x) = sum_mu U'_G(x,mu) U(x,mu)^+ + U'_G(x-mu,mu)^+ U(x-mu,mu),
//   C = Delta - Delta^+ - Tr(Delta - Delta^+)/3,  k(x) = exp(alpha/2 C) on the domain,
// a step accepted when it lowers eq. relgf (G -> G k), and at the end g = G^(1/2), the
// pair (U^g, U'^(g^-1)). The domain is the block-interior sites (local coordinates
// 1 .. b_mu - 2). The exponential is a scaled Taylor series squared back; the square
// root the Denman-Beavers iteration; both end with a projection onto SU(3).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace psms {

struct GfGeo {
  int L[4], b[4];
  int V;
};

using C3 = SU3<double>;

__device__ __forceinline__ C3 ld3(const double* __restrict__ p) {
  C3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) m.m[k / 3][k % 3] = {p[2 * k], p[2 * k + 1]};
  return m;
}
__device__ __forceinline__ void st3(double* __restrict__ p, const C3& m) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    p[2 * k] = m.m[k / 3][k % 3].re;
    p[2 * k + 1] = m.m[k / 3][k % 3].im;
  }
}
__device__ __forceinline__ C3 eye3() {
  C3 m;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) m.m[i][j] = {i == j ? 1.0 : 0.0, 0.0};
  return m;
}
// A B (da: A^+ instead of A; db: B^+ instead of B)
__device__ __forceinline__ C3 mul3(const C3& A, const C3& B, bool da = false, bool db = false) {
  C3 o;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        cx<double> a = da ? cx<double>{A.m[k][i].re, -A.m[k][i].im} : A.m[i][k];
        cx<double> b = db ? cx<double>{B.m[j][k].re, -B.m[j][k].im} : B.m[k][j];
        s = s + cmul(a, b);
      }
      o.m[i][j] = s;
    }
  return o;
}
__device__ __forceinline__ C3 add3(const C3& A, const C3& B, double sb = 1.0) {
  C3 o;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) o.m[i][j] = {A.m[i][j].re + sb * B.m[i][j].re, A.m[i][j].im + sb * B.m[i][j].im};
  return o;
}
__device__ __forceinline__ C3 scale3(const C3& A, double s) {
  C3 o;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) o.m[i][j] = {s * A.m[i][j].re, s * A.m[i][j].im};
  return o;
}
// the nearest SU(3) matrix in the sense used for the links: Gram-Schmidt on rows 0, 1,
// row 2 = conj(row 0 x row 1)
__device__ C3 project_su3(const C3& A) {
  C3 o = A;
  double n0 = 0.0;
  for (int j = 0; j < 3; ++j) n0 += o.m[0][j].re * o.m[0][j].re + o.m[0][j].im * o.m[0][j].im;
  n0 = 1.0 / sqrt(n0);
  for (int j = 0; j < 3; ++j) o.m[0][j] = scale(n0, o.m[0][j]);
  cx<double> d = {0.0, 0.0};
  for (int j = 0; j < 3; ++j) d = d + cjmul(o.m[0][j], o.m[1][j]);
  for (int j = 0; j < 3; ++j) o.m[1][j] = o.m[1][j] - cmul(d, o.m[0][j]);
  double n1 = 0.0;
  for (int j = 0; j < 3; ++j) n1 += o.m[1][j].re * o.m[1][j].re + o.m[1][j].im * o.m[1][j].im;
  n1 = 1.0 / sqrt(n1);
  for (int j = 0; j < 3; ++j) o.m[1][j] = scale(n1, o.m[1][j]);
  for (int j = 0; j < 3; ++j) {
    const int a = (j + 1) % 3, b = (j + 2) % 3;
    cx<double> c = cmul(o.m[0][a], o.m[1][b]) - cmul(o.m[0][b], o.m[1][a]);
    o.m[2][j] = {c.re, -c.im};
  }
  return o;
}
// exp(X) for a traceless anti-Hermitian X: X / 2^s with |X / 2^s|_F <= 1/2, Taylor to
// degree 16 (remainder below 1e-18), squared s times, projected onto SU(3).
__device__ C3 exp_ah(const C3& X) {
  double nf = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) nf += X.m[i][j].re * X.m[i][j].re + X.m[i][j].im * X.m[i][j].im;
  nf = sqrt(nf);
  int s = 0;
  while (nf > 0.5 && s < 60) {
    nf *= 0.5;
    ++s;
  }
  const C3 Y = scale3(X, ldexp(1.0, -s));
  C3 E = eye3();
  for (int k = 16; k >= 1; --k) E = add3(eye3(), scale3(mul3(Y, E), 1.0 / k));  // Horner: 1 + Y/k (...)
  for (int q = 0; q < s; ++q) E = mul3(E, E);
  return project_su3(E);
}
// inverse of a 3x3 complex matrix by its adjugate
__device__ C3 inv3(const C3& A) {
  C3 adj;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
      adj.m[i][j] = cmul(A.m[r0][c0], A.m[r1][c1]) - cmul(A.m[r0][c1], A.m[r1][c0]);
    }
  cx<double> det = cmul(A.m[0][0], adj.m[0][0]) + cmul(A.m[0][1], adj.m[1][0]) + cmul(A.m[0][2], adj.m[2][0]);
  const double dn = det.re * det.re + det.im * det.im;
  const cx<double> id = {det.re / dn, -det.im / dn};
  C3 o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.m[i][j] = cmul(adj.m[i][j], id);
  return o;
}
// principal square root (Denman-Beavers: Y -> (Y + Z^-1)/2, Z -> (Z + Y^-1)/2 from Y = G,
// Z = 1), projected onto SU(3)
__device__ C3 sqrt_su3(const C3& G) {
  C3 Y = G, Z = eye3();
  for (int it = 0; it < 12; ++it) {
    const C3 Yi = inv3(Y), Zi = inv3(Z);
    Y = scale3(add3(Y, Zi), 0.5);
    Z = scale3(add3(Z, Yi), 0.5);
  }
  return project_su3(Y);
}

__device__ __forceinline__ void coords_of(const GfGeo& g, int lex, int (&x)[4]) {
  int r = lex;
  x[3] = r % g.L[3]; r /= g.L[3];
  x[2] = r % g.L[2]; r /= g.L[2];
  x[1] = r % g.L[1]; x[0] = r / g.L[1];
}
__device__ __forceinline__ int lex_of(const GfGeo& g, const int (&x)[4]) {
  return ((x[0] * g.L[1] + x[1]) * g.L[2] + x[2]) * g.L[3] + x[3];
}
__device__ __forceinline__ int shifted(const GfGeo& g, const int (&x)[4], int mu, int d) {
  int y[4] = {x[0], x[1], x[2], x[3]};
  y[mu] = (y[mu] + d + g.L[mu]) % g.L[mu];
  return lex_of(g, y);
}
__device__ __forceinline__ bool in_domain(const GfGeo& g, const int (&x)[4]) {
  bool in = true;
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int l = x[m] % g.b[m];
    in = in && l >= 1 && l <= g.b[m] - 2;
  }
  return in;
}

// fixed-order sum of one value per thread into part[blockIdx.x]
__device__ __forceinline__ void block_sum(double v, double* __restrict__ part) {
  __shared__ double sm[256];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] += sm[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

// internal FP64 links (layout g) -> boundary layout
__global__ void k_gf_unpack(Geo g, const double2* __restrict__ Lint, double* __restrict__ U, int V) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int p, s;
  lex_to_internal(g, lex, p, s);
  const size_t Vh = g.Vh;
  for (int mu = 0; mu < 4; ++mu)
    for (int k = 0; k < 9; ++k) {
      const double2 v = Lint[size_t(p * 4 + mu) * 9 * Vh + k * Vh + s];
      U[(size_t(lex) * 4 + mu) * 18 + 2 * k] = v.x;
      U[(size_t(lex) * 4 + mu) * 18 + 2 * k + 1] = v.y;
    }
}

// G = 1 everywhere
__global__ void k_gf_eye(double* __restrict__ G, int V) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < V) st3(G + size_t(x) * 18, eye3());
}

// Delta, C and theta on the current pair; K = exp(half_alpha C) on the domain, 1 elsewhere;
// theta summed over the domain sites of the workgroup
__global__ void __launch_bounds__(256) k_gf_step(GfGeo g, const double* __restrict__ U, const double* __restrict__ Upc,
                                                 double* __restrict__ K, double half_alpha, double* __restrict__ theta_part) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  double th = 0.0;
  if (lex < g.V) {
    int x[4];
    coords_of(g, lex, x);
    C3 k = eye3();
    if (in_domain(g, x)) {
      C3 D;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) D.m[i][j] = {0.0, 0.0};
      for (int mu = 0; mu < 4; ++mu) {
        const size_t f = (size_t(lex) * 4 + mu) * 18;
        D = add3(D, mul3(ld3(Upc + f), ld3(U + f), false, true));
        const size_t bw = (size_t(shifted(g, x, mu, -1)) * 4 + mu) * 18;
        D = add3(D, mul3(ld3(Upc + bw), ld3(U + bw), true, false));
      }
      C3 C;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) C.m[i][j] = {D.m[i][j].re - D.m[j][i].re, D.m[i][j].im + D.m[j][i].im};
      const double tr = (C.m[0][0].im + C.m[1][1].im + C.m[2][2].im) / 3.0;  // C is anti-Hermitian: real diagonal 0
      for (int i = 0; i < 3; ++i) C.m[i][i].im -= tr;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) th += C.m[i][j].re * C.m[i][j].re + C.m[i][j].im * C.m[i][j].im;
      k = exp_ah(scale3(C, half_alpha));
    }
    st3(K + size_t(lex) * 18, k);
  }
  block_sum(th, theta_part);
}

// trial field U'_t(x,mu) = K(x)^+ U'_G(x,mu) K(x+mu); sum of Re Tr(U^+ U'_t) per workgroup
__global__ void __launch_bounds__(256) k_gf_trial(GfGeo g, const double* __restrict__ U, const double* __restrict__ Upc,
                                                  const double* __restrict__ K, double* __restrict__ Upt,
                                                  double* __restrict__ f_part) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (lex < g.V) {
    int x[4];
    coords_of(g, lex, x);
    const C3 kx = ld3(K + size_t(lex) * 18);
    for (int mu = 0; mu < 4; ++mu) {
      const size_t f = (size_t(lex) * 4 + mu) * 18;
      const C3 ky = ld3(K + size_t(shifted(g, x, mu, +1)) * 18);
      const C3 t = mul3(mul3(kx, ld3(Upc + f), true, false), ky);
      st3(Upt + f, t);
      const C3 u = ld3(U + f);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc += u.m[i][j].re * t.m[i][j].re + u.m[i][j].im * t.m[i][j].im;
    }
  }
  block_sum(acc, f_part);
}

// sum of Re Tr(U^+ U') per workgroup
__global__ void __launch_bounds__(256) k_gf_overlap(GfGeo g, const double* __restrict__ U, const double* __restrict__ Up,
                                                    double* __restrict__ f_part) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (lex < g.V)
    for (int e = 0; e < 4 * 18; e += 2) {
      const size_t o = size_t(lex) * 72 + e;
      acc += U[o] * Up[o] + U[o + 1] * Up[o + 1];
    }
  block_sum(acc, f_part);
}

// G <- G K (an accepted step)
__global__ void k_gf_accept(GfGeo g, double* __restrict__ G, const double* __restrict__ K) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x < g.V) st3(G + size_t(x) * 18, mul3(ld3(G + size_t(x) * 18), ld3(K + size_t(x) * 18)));
}

// g = G^(1/2) on the domain, 1 elsewhere
__global__ void k_gf_sqrt(GfGeo g, const double* __restrict__ G, double* __restrict__ gout) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= g.V) return;
  int x[4];
  coords_of(g, lex, x);
  st3(gout + size_t(lex) * 18, in_domain(g, x) ? sqrt_su3(ld3(G + size_t(lex) * 18)) : eye3());
}

// (U^g, U'^(g^-1)): U(x,mu) -> g(x) U g(x+mu)^+, U'(x,mu) -> g(x)^+ U' g(x+mu)
__global__ void k_gf_transform(GfGeo g, const double* __restrict__ gf, const double* __restrict__ U,
                               const double* __restrict__ Up, double* __restrict__ Ug, double* __restrict__ Upg) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= g.V) return;
  int x[4];
  coords_of(g, lex, x);
  const C3 gx = ld3(gf + size_t(lex) * 18);
  for (int mu = 0; mu < 4; ++mu) {
    const size_t f = (size_t(lex) * 4 + mu) * 18;
    const C3 gy = ld3(gf + size_t(shifted(g, x, mu, +1)) * 18);
    st3(Ug + f, mul3(mul3(gx, ld3(U + f)), gy, false, true));
    st3(Upg + f, mul3(mul3(gx, ld3(Up + f), true, false), gy));
  }
}

static GfGeo gf_geo(const Geo& g) {
  GfGeo o;
  o.V = 2 * g.Vh;
  for (int m = 0; m < 4; ++m) {
    o.L[m] = g.L[m];
    o.b[m] = g.b[m];
  }
  return o;
}
static int gf_blocks(const Geo& g) { return (2 * g.Vh + 255) / 256; }
int gf_partials(const Geo& g) { return gf_blocks(g); }

void launch_gf_unpack(hipStream_t st, const Geo& g, const void* links_f64, double* U) {
  hipLaunchKernelGGL(k_gf_unpack, dim3(gf_blocks(g)), dim3(256), 0, st, g, (const double2*)links_f64, U, 2 * g.Vh);
}
void launch_gf_eye(hipStream_t st, const Geo& g, double* G) {
  hipLaunchKernelGGL(k_gf_eye, dim3(gf_blocks(g)), dim3(256), 0, st, G, 2 * g.Vh);
}
void launch_gf_step(hipStream_t st, const Geo& g, const double* U, const double* Upc, double* K, double half_alpha,
                    double* theta_part) {
  hipLaunchKernelGGL(k_gf_step, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), U, Upc, K, half_alpha, theta_part);
}
void launch_gf_trial(hipStream_t st, const Geo& g, const double* U, const double* Upc, const double* K, double* Upt,
                     double* f_part) {
  hipLaunchKernelGGL(k_gf_trial, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), U, Upc, K, Upt, f_part);
}
void launch_gf_overlap(hipStream_t st, const Geo& g, const double* U, const double* Up, double* f_part) {
  hipLaunchKernelGGL(k_gf_overlap, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), U, Up, f_part);
}
void launch_gf_accept(hipStream_t st, const Geo& g, double* G, const double* K) {
  hipLaunchKernelGGL(k_gf_accept, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), G, K);
}
void launch_gf_finish(hipStream_t st, const Geo& g, const double* G, double* gout, const double* U, const double* Up,
                      double* Ug, double* Upg) {
  hipLaunchKernelGGL(k_gf_sqrt, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), G, gout);
  hipLaunchKernelGGL(k_gf_transform, dim3(gf_blocks(g)), dim3(256), 0, st, gf_geo(g), (const double*)gout, U, Up, Ug,
                     Upg);
}

// ----------------------------------------------------------------- link-field merges
// The hierarchy of filters combines fields block by block: out(x, mu) = U'(x, mu) when the
// link lies inside a block (both ends in the block x // b) whose accept flag is set, else U.
__device__ __forceinline__ int block_lex(const GfGeo& g, const int (&x)[4]) {
  int B[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) B[m] = x[m] / g.b[m];
  return ((B[0] * (g.L[1] / g.b[1]) + B[1]) * (g.L[2] / g.b[2]) + B[2]) * (g.L[3] / g.b[3]) + B[3];
}

__global__ void k_merge_links(GfGeo g, const int* __restrict__ accept, const double* __restrict__ U,
                              const double* __restrict__ Up, double* __restrict__ out) {
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= g.V) return;
  int x[4];
  coords_of(g, lex, x);
  const int bx = block_lex(g, x);
  for (int mu = 0; mu < 4; ++mu) {
    int y[4] = {x[0], x[1], x[2], x[3]};
    y[mu] = (y[mu] + 1) % g.L[mu];
    const bool take = block_lex(g, y) == bx && accept[bx];
    const size_t f = (size_t(lex) * 4 + mu) * 18;
    for (int e = 0; e < 18; ++e) out[f + e] = take ? Up[f + e] : U[f + e];
  }
}

// max |U' - U| over the links that leave their block (per workgroup)
__global__ void __launch_bounds__(256) k_change_across(GfGeo g, const double* __restrict__ U,
                                                       const double* __restrict__ Up, double* __restrict__ part) {
  __shared__ double sm[256];
  const int lex = blockIdx.x * blockDim.x + threadIdx.x;
  double m = 0.0;
  if (lex < g.V) {
    int x[4];
    coords_of(g, lex, x);
    const int bx = block_lex(g, x);
    for (int mu = 0; mu < 4; ++mu) {
      int y[4] = {x[0], x[1], x[2], x[3]};
      y[mu] = (y[mu] + 1) % g.L[mu];
      if (block_lex(g, y) == bx) continue;
      const size_t f = (size_t(lex) * 4 + mu) * 18;
      for (int e = 0; e < 18; ++e) {
        const double d = fabs(Up[f + e] - U[f + e]);
        m = (d > m || d != d) ? d : m;
      }
    }
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double d = sm[threadIdx.x + o];
      sm[threadIdx.x] = (d > sm[threadIdx.x] || d != d) ? d : sm[threadIdx.x];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

void launch_merge_links(hipStream_t st, const Geo& g, const int* b, const int* accept, const double* U, const double* Up,
                        double* out) {
  GfGeo gg = gf_geo(g);
  for (int m = 0; m < 4; ++m) gg.b[m] = b[m];
  hipLaunchKernelGGL(k_merge_links, dim3(gf_blocks(g)), dim3(256), 0, st, gg, accept, U, Up, out);
}

void launch_change_across(hipStream_t st, const Geo& g, const int* b, const double* U, const double* Up, double* part) {
  GfGeo gg = gf_geo(g);
  for (int m = 0; m < 4; ++m) gg.b[m] = b[m];
  hipLaunchKernelGGL(k_change_across, dim3(gf_blocks(g)), dim3(256), 0, st, gg, U, Up, part);
}

}  // namespace psms
