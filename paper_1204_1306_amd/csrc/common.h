// Device-side building blocks of the Wilson-Dirac hot path on gfx950:
// complex arithmetic, spinor/link storage formats, the block-major even-odd
// site layout and the spin-projected nearest-neighbour hop.
//
// Operator (eq. Dw, Sec. 5, rescaled): D = 1 - kappa H with
//   H psi(x) = sum_mu U(x,mu)(1-gamma_mu) psi(x+mu) + U(x-mu,mu)^+ (1+gamma_mu) psi(x-mu),
// antiperiodic in time (Sec. 6). Chiral gamma basis:
//   gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]], gamma_5 = diag(1,1,-1,-1).
// (1 -+ gamma_mu) has rank two, so each hop projects the spinor to two spin
// components, multiplies them by the 3x3 link and rebuilds the lower half.
//
// Internal layout (sites innermost, one component plane per storage unit):
//   site (parity p, index s) with s = blk * Vbh + i, blk = colour * nblk_c + (lexB >> 1),
//   i = locallex >> 1 (blocks sorted black first as in eq. domdec; even-odd inside blocks).
//   spinor field: [rhs][p][unit k][Vh]; link field: [p][mu][unit k][Vh] holding U(x,mu).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psms {

// ----------------------------------------------------------------- complex
template <class T> struct cx { T re, im; };

template <class T> __host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T> __host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <class T> __host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T> __host__ __device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.im, a.re}; }
template <class T> __host__ __device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.im, -a.re}; }
template <class T> __host__ __device__ __forceinline__ cx<T> scale(T s, cx<T> a) { return {s * a.re, s * a.im}; }

template <class T> struct Spinor { cx<T> v[4][3]; };   // [spin][colour]
template <class T> struct SU3 { cx<T> m[3][3]; };      // [row][col]

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Row 2 of an SU(3) matrix from rows 0 and 1, times f: f conj(row0 x row1), each
// component one multiply and three fused multiply-adds.
template <class T> __device__ __forceinline__ void su3_row2(SU3<T>& u, T f) {
  const cx<T>(&r0)[3] = u.m[0];
  const cx<T>(&r1)[3] = u.m[1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int i = (c + 1) % 3, k = (c + 2) % 3;  // component c of r0 x r1 = r0[i] r1[k] - r0[k] r1[i]
    T re = r0[i].re * r1[k].re, im = r0[i].re * r1[k].im;
    re = fmadd(-r0[i].im, r1[k].im, re);
    re = fmadd(-r0[k].re, r1[i].re, re);
    re = fmadd(r0[k].im, r1[i].im, re);
    im = fmadd(r0[i].im, r1[k].re, im);
    im = fmadd(-r0[k].re, r1[i].im, im);
    im = fmadd(-r0[k].im, r1[i].re, im);
    u.m[2][c] = {f * re, -(f * im)};
  }
}
template <class T> struct Half { cx<T> h[2][3]; };     // projected two-spin vector

template <class T> __host__ __device__ __forceinline__ void zero(Spinor<T>& s) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) s.v[a][c] = {T(0), T(0)};
}

// ----------------------------------------------------------------- bf16
// Round-to-nearest-even float -> bfloat16 from the IEEE-754 binary32 layout:
// keep the top 16 bits, adding half an ulp of bf16 plus the tie-break bit.
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return uint16_t((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__host__ __device__ __forceinline__ float bf16_to_f32(uint32_t h) { return __builtin_bit_cast(float, h << 16); }
// Two floats to a packed bfloat16 pair (lo, hi) with gfx950's conversion instruction: one
// instruction per pair, but its results differ from f32_to_bf16 on some inputs, so it is
// used only where the rounding of the last bit does not matter (the Schwarz
// preconditioner's own fields); every other BF16 store rounds to nearest even exactly.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack2(float lo, float hi) {
  const bf16x2_t v = {__bf16(lo), __bf16(hi)};
  return __builtin_bit_cast(uint32_t, v);
}

// Non-temporal 16-byte accesses (streamed data that is not read again soon: the
// output of a full-lattice stencil), so the L2 keeps the neighbour spinors.
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
template <class V> __device__ __forceinline__ void nt_st(V* p, V v) {
  static_assert(sizeof(V) == 16, "16-byte storage units");
  nt_u4 n;
  __builtin_memcpy(&n, &v, 16);
  __builtin_nontemporal_store(n, reinterpret_cast<nt_u4*>(p));
}

// ----------------------------------------------------------------- storage formats
// Spinor storage: F64 = 12 double2 planes, F32 = 6 float4 planes, BF16 = 3 uint4 planes.
enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

struct StF64 {
  using unit = double2;
  using real = double;
  static constexpr int NC = 12;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      double2 d = p[k * Vh + s];
      o.v[k / 3][k % 3] = {T(d.x), T(d.y)};
    }
  }
  template <class T> __device__ __forceinline__ static void store(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k * Vh + s] = make_double2(double(o.v[k / 3][k % 3].re), double(o.v[k / 3][k % 3].im));
  }
  template <class T> __device__ __forceinline__ static void store_nt(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 12; ++k) nt_st(p + k * Vh + s, make_double2(double(o.v[k / 3][k % 3].re), double(o.v[k / 3][k % 3].im)));
  }
};

struct StF32 {
  using unit = float4;
  using real = float;
  static constexpr int NC = 6;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float4 d = p[k * Vh + s];
      o.v[(2 * k) / 3][(2 * k) % 3] = {T(d.x), T(d.y)};
      o.v[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(d.z), T(d.w)};
    }
  }
  template <class T> __device__ __forceinline__ static void store(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cx<T> a = o.v[(2 * k) / 3][(2 * k) % 3], b = o.v[(2 * k + 1) / 3][(2 * k + 1) % 3];
      p[k * Vh + s] = make_float4(float(a.re), float(a.im), float(b.re), float(b.im));
    }
  }
  template <class T> __device__ __forceinline__ static void store_nt(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      cx<T> a = o.v[(2 * k) / 3][(2 * k) % 3], b = o.v[(2 * k + 1) / 3][(2 * k + 1) % 3];
      nt_st(p + k * Vh + s, make_float4(float(a.re), float(a.im), float(b.re), float(b.im)));
    }
  }
};

struct StBF16 {
  using unit = uint4;
  using real = float;
  static constexpr int NC = 3;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint4 d = p[k * Vh + s];
      uint32_t w[4] = {d.x, d.y, d.z, d.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int e = 4 * k + j;
        o.v[e / 3][e % 3] = {T(bf16_to_f32(w[j] & 0xffffu)), T(bf16_to_f32(w[j] >> 16))};
      }
    }
  }
  template <class T> __device__ __forceinline__ static void store(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int e = 4 * k + j;
        w[j] = uint32_t(f32_to_bf16(float(o.v[e / 3][e % 3].re))) | (uint32_t(f32_to_bf16(float(o.v[e / 3][e % 3].im))) << 16);
      }
      p[k * Vh + s] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }
  template <class T> __device__ __forceinline__ static void store_nt(unit* __restrict__ p, size_t Vh, int s, const Spinor<T>& o) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        int e = 4 * k + j;
        w[j] = uint32_t(f32_to_bf16(float(o.v[e / 3][e % 3].re))) | (uint32_t(f32_to_bf16(float(o.v[e / 3][e % 3].im))) << 16);
      }
      nt_st(p + k * Vh + s, make_uint4(w[0], w[1], w[2], w[3]));
    }
  }
};

// Link storage: F64 = 9 double2 planes; F32C12 = rows 0 and 1 as 3 float4 planes,
// row 2 rebuilt as conj(row0 x row1) (valid for SU(3) links only).
struct LkF64 {
  using unit = double2;
  static constexpr int NC = 9;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, SU3<T>& u) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      double2 d = p[k * Vh + s];
      u.m[k / 3][k % 3] = {T(d.x), T(d.y)};
    }
  }
};

struct LkF32C12 {
  using unit = float4;
  static constexpr int NC = 3;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, SU3<T>& u) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float4 d = p[k * Vh + s];
      u.m[(2 * k) / 3][(2 * k) % 3] = {T(d.x), T(d.y)};
      u.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(d.z), T(d.w)};
    }
    su3_row2(u, T(1));
  }
};

// F32F18: all 18 reals in FP32, for links that are not SU(3) (the fields between U and U'
// of an interpolated estimate): 5 float4 planes, complex entries (2k, 2k + 1) in plane k,
// entry 8 and a zero pad in plane 4.
struct LkF32F18 {
  using unit = float4;
  static constexpr int NC = 5;
  template <class T> __device__ __forceinline__ static void load(const unit* __restrict__ p, size_t Vh, int s, SU3<T>& u) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float4 d = p[k * Vh + s];
      u.m[(2 * k) / 3][(2 * k) % 3] = {T(d.x), T(d.y)};
      u.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(d.z), T(d.w)};
    }
    float4 d = p[4 * Vh + s];
    u.m[2][2] = {T(d.x), T(d.y)};
  }
};

// ----------------------------------------------------------------- geometry
struct Geo {
  int L[4], b[4], NB[4];
  int sB[4], sl[4];       // lexicographic strides of block coords and local coords
  int Vh, Vbh, nblk, nblk_c;
  int apbc;
  int ob[4];               // outer (Dirichlet) block extent of the recursive decomposition, 0: none
  const uint32_t* lcoord;  // [2][Vbh] local coords of (parity, i), 8 bits each
  const uint32_t* bcoord;  // [nblk] block coords of blk, 8 bits each
  const int* border;       // [nblk] the order in which the stencil visits blocks (black, then its white neighbour)
};

// Everything the stencil needs about one site.
struct SiteInfo {
  int l[4], B[4];
  int locallex, lexB, colour;
};

__device__ __forceinline__ void site_info(const Geo& g, int p, int s, SiteInfo& si) {
  int blk = s / g.Vbh;
  int i = s - blk * g.Vbh;
  uint32_t lc = g.lcoord[p * g.Vbh + i];
  uint32_t bc = g.bcoord[blk];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    si.l[m] = (lc >> (8 * m)) & 255;
    si.B[m] = (bc >> (8 * m)) & 255;
  }
  si.colour = blk >= g.nblk_c ? 1 : 0;
  si.locallex = 2 * i + (si.l[3] & 1);
  si.lexB = 2 * (blk - si.colour * g.nblk_c) + (si.B[3] & 1);
}

// Neighbour x + dir*mu (dir = +1 or -1). Returns its index within the opposite
// parity, whether the hop leaves the block and the boundary sign (-1 across the
// time boundary with antiperiodic fermions).
struct Nbr {
  int s;
  bool cross;
  float sign;
};

__device__ __forceinline__ Nbr neighbour(const Geo& g, const SiteInfo& si, int mu, int dir) {
  Nbr n;
  int ll = si.locallex, lb = si.lexB, col = si.colour;
  int lm = si.l[mu] + dir;
  n.sign = 1.f;
  if (lm >= 0 && lm < g.b[mu]) {
    ll += dir * g.sl[mu];
    n.cross = false;
  } else {
    n.cross = true;
    ll -= dir * (g.b[mu] - 1) * g.sl[mu];
    int Bm = si.B[mu] + dir;
    if (Bm < 0) {
      lb += (g.NB[mu] - 1) * g.sB[mu];
      if (mu == 0 && g.apbc) n.sign = -1.f;
    } else if (Bm >= g.NB[mu]) {
      lb -= (g.NB[mu] - 1) * g.sB[mu];
      if (mu == 0 && g.apbc) n.sign = -1.f;
    } else {
      lb += dir * g.sB[mu];
    }
    col ^= 1;
  }
  n.s = (col * g.nblk_c + (lb >> 1)) * g.Vbh + (ll >> 1);
  return n;
}

// Read-only view of site q of a [12][N] LDS field as a spinor (p.v[spin][colour]), so
// a hop reads each component where it uses it instead of copying the spinor first.
template <class T, int N> struct LdsSpinor {
  struct Row {
    const cx<T> (*f)[N];
    int q, i;
    __device__ __forceinline__ cx<T> operator[](int c) const { return f[3 * i + c][q]; }
  };
  struct Rows {
    const cx<T> (*f)[N];
    int q;
    __device__ __forceinline__ Row operator[](int i) const { return {f, q, i}; }
  };
  Rows v;
};

// ----------------------------------------------------------------- SU(3) x vector

// o = U v and o = U^+ v. Each real component is one chain of a multiply and five fused
// multiply-adds (12 operations per complex entry, against 16 for three complex products
// summed).
template <class T> __device__ __forceinline__ void su3_mul(const SU3<T>& u, const cx<T> (&v)[3], cx<T> (&o)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T re = u.m[a][0].re * v[0].re, im = u.m[a][0].re * v[0].im;
    re = fmadd(-u.m[a][0].im, v[0].im, re);
    im = fmadd(u.m[a][0].im, v[0].re, im);
#pragma unroll
    for (int b = 1; b < 3; ++b) {
      re = fmadd(u.m[a][b].re, v[b].re, re);
      re = fmadd(-u.m[a][b].im, v[b].im, re);
      im = fmadd(u.m[a][b].re, v[b].im, im);
      im = fmadd(u.m[a][b].im, v[b].re, im);
    }
    o[a] = {re, im};
  }
}
template <class T> __device__ __forceinline__ void su3_dag_mul(const SU3<T>& u, const cx<T> (&v)[3], cx<T> (&o)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T re = u.m[0][a].re * v[0].re, im = u.m[0][a].re * v[0].im;
    re = fmadd(u.m[0][a].im, v[0].im, re);
    im = fmadd(-u.m[0][a].im, v[0].re, im);
#pragma unroll
    for (int b = 1; b < 3; ++b) {
      re = fmadd(u.m[b][a].re, v[b].re, re);
      re = fmadd(u.m[b][a].im, v[b].im, re);
      im = fmadd(u.m[b][a].re, v[b].im, im);
      im = fmadd(-u.m[b][a].im, v[b].re, im);
    }
    o[a] = {re, im};
  }
}

// The same products as sums of three complex products: more operations, but shorter
// dependency chains, which keeps fewer values live where registers are the limit.
template <class T> __device__ __forceinline__ void su3_mul_sum(const SU3<T>& u, const cx<T> (&v)[3], cx<T> (&o)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = cmul(u.m[a][0], v[0]) + cmul(u.m[a][1], v[1]) + cmul(u.m[a][2], v[2]);
}
template <class T> __device__ __forceinline__ void su3_dag_mul_sum(const SU3<T>& u, const cx<T> (&v)[3], cx<T> (&o)[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) o[a] = cjmul(u.m[0][a], v[0]) + cjmul(u.m[1][a], v[1]) + cjmul(u.m[2][a], v[2]);
}

// acc += c * U(x,mu) (1 - gamma_mu) psi   (psi = psi(x+mu), c includes the boundary sign).
// P is Spinor<T> or any view whose p.v[spin][colour] yields cx<T>.
template <class T, class P> __device__ __forceinline__ void hop_fwd(int mu, const SU3<T>& U, const P& p, T c, Spinor<T>& acc) {
  cx<T> h0[3], h1[3], u0[3], u1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    switch (mu) {
      case 0: h0[a] = p.v[0][a] + p.v[2][a]; h1[a] = p.v[1][a] + p.v[3][a]; break;
      case 1: h0[a] = p.v[0][a] + times_i(p.v[3][a]); h1[a] = p.v[1][a] + times_i(p.v[2][a]); break;
      case 2: h0[a] = p.v[0][a] + p.v[3][a]; h1[a] = p.v[1][a] - p.v[2][a]; break;
      default: h0[a] = p.v[0][a] + times_i(p.v[2][a]); h1[a] = p.v[1][a] - times_i(p.v[3][a]); break;
    }
  }
  su3_mul(U, h0, u0);
  su3_mul(U, h1, u1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    u0[a] = scale(c, u0[a]);
    u1[a] = scale(c, u1[a]);
    acc.v[0][a] = acc.v[0][a] + u0[a];
    acc.v[1][a] = acc.v[1][a] + u1[a];
    switch (mu) {
      case 0: acc.v[2][a] = acc.v[2][a] + u0[a]; acc.v[3][a] = acc.v[3][a] + u1[a]; break;
      case 1: acc.v[2][a] = acc.v[2][a] + times_mi(u1[a]); acc.v[3][a] = acc.v[3][a] + times_mi(u0[a]); break;
      case 2: acc.v[2][a] = acc.v[2][a] - u1[a]; acc.v[3][a] = acc.v[3][a] + u0[a]; break;
      default: acc.v[2][a] = acc.v[2][a] + times_mi(u0[a]); acc.v[3][a] = acc.v[3][a] + times_i(u1[a]); break;
    }
  }
}

// The backward hop in two halves, so that the site that owns the link and the spinor
// can compute the colour part and hand it to its +mu neighbour:
//   bwd_half:  w0, w1 = U^+ times the two independent rows of (1 + gamma_mu) psi;
//   bwd_recon: acc += c * (the full spinor those two rows determine).
template <class T, class P>
__device__ __forceinline__ void bwd_half(int mu, const SU3<T>& U, const P& p, cx<T> (&w0)[3], cx<T> (&w1)[3]) {
  cx<T> h0[3], h1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    switch (mu) {
      case 0: h0[a] = p.v[0][a] - p.v[2][a]; h1[a] = p.v[1][a] - p.v[3][a]; break;
      case 1: h0[a] = p.v[0][a] + times_mi(p.v[3][a]); h1[a] = p.v[1][a] + times_mi(p.v[2][a]); break;
      case 2: h0[a] = p.v[0][a] - p.v[3][a]; h1[a] = p.v[1][a] + p.v[2][a]; break;
      default: h0[a] = p.v[0][a] + times_mi(p.v[2][a]); h1[a] = p.v[1][a] + times_i(p.v[3][a]); break;
    }
  }
  su3_dag_mul(U, h0, w0);
  su3_dag_mul(U, h1, w1);
}
template <class T>
__device__ __forceinline__ void bwd_recon(int mu, cx<T> (&w0)[3], cx<T> (&w1)[3], T c, Spinor<T>& acc) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w0[a] = scale(c, w0[a]);
    w1[a] = scale(c, w1[a]);
    acc.v[0][a] = acc.v[0][a] + w0[a];
    acc.v[1][a] = acc.v[1][a] + w1[a];
    switch (mu) {
      case 0: acc.v[2][a] = acc.v[2][a] - w0[a]; acc.v[3][a] = acc.v[3][a] - w1[a]; break;
      case 1: acc.v[2][a] = acc.v[2][a] + times_i(w1[a]); acc.v[3][a] = acc.v[3][a] + times_i(w0[a]); break;
      case 2: acc.v[2][a] = acc.v[2][a] + w1[a]; acc.v[3][a] = acc.v[3][a] - w0[a]; break;
      default: acc.v[2][a] = acc.v[2][a] + times_i(w0[a]); acc.v[3][a] = acc.v[3][a] - times_i(w1[a]); break;
    }
  }
}

// acc += c * U(x-mu,mu)^+ (1 + gamma_mu) psi   (psi = psi(x-mu))
template <class T, class P> __device__ __forceinline__ void hop_bwd(int mu, const SU3<T>& U, const P& p, T c, Spinor<T>& acc) {
  cx<T> w0[3], w1[3];
  bwd_half(mu, U, p, w0, w1);
  bwd_recon(mu, w0, w1, c, acc);
}

// ----------------------------------------------------------------- reductions
// Wave64 sum with DPP-free shuffles (__shfl_xor), deterministic order.
template <class T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The same sum through the data-parallel-primitive (DPP) lane network, for waves
// whose 64 lanes are all active: xor-1 and xor-2 swaps inside quads, then the
// half-row and row mirrors give every lane of a 16-lane row the row's sum (each step
// pairs lanes holding equal partial sums, so the mirrors act as xor-4 and xor-8);
// the four row sums are then added in a fixed order from lanes 0, 16, 32 and 48.
// No LDS round trips, deterministic, and the result is wave-uniform.
template <int CTRL> __device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]: xor 1
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]: xor 2
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}
// Every FP64 wave sum of the library runs on full waves (all call sites reduce after
// workgroup-uniform loops), so the overload for double takes the DPP form.
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_dpp(v); }

// ----------------------------------------------------------------- site index conversion
// Internal (parity, s) of the site with coordinates x.
__device__ __forceinline__ void coords_to_internal(const Geo& g, const int (&x)[4], int& p, int& s) {
  int B[4], l[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    B[m] = x[m] / g.b[m];
    l[m] = x[m] - B[m] * g.b[m];
  }
  int lexB = ((B[0] * g.NB[1] + B[1]) * g.NB[2] + B[2]) * g.NB[3] + B[3];
  int col = (B[0] + B[1] + B[2] + B[3]) & 1;
  int ll = ((l[0] * g.b[1] + l[1]) * g.b[2] + l[2]) * g.b[3] + l[3];
  p = (x[0] + x[1] + x[2] + x[3]) & 1;
  s = (col * g.nblk_c + (lexB >> 1)) * g.Vbh + (ll >> 1);
}

// Internal (parity, s) of a lexicographic site.
__device__ __forceinline__ void lex_to_internal(const Geo& g, int lex, int& p, int& s) {
  int x[4];
  int r = lex;
  x[3] = r % g.L[3]; r /= g.L[3];
  x[2] = r % g.L[2]; r /= g.L[2];
  x[1] = r % g.L[1]; x[0] = r / g.L[1];
  coords_to_internal(g, x, p, s);
}

}  // namespace psms
