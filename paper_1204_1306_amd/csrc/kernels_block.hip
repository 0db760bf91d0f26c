// Block solves for the Schwarz preconditioner and the Dirichlet block inverses
// D_bb^-1, D_ww^-1 of the Schur complement (eq. ddfactor). One workgroup owns one
// block of one right-hand side: all blocks of a colour, all right-hand sides and
// all proposals run in a single launch. The block operator D_b is the principal
// sub-matrix of D on the block (hops leaving the block are dropped: Dirichlet).
// Minimal-residual iteration; the workgroup reduces its own inner products, so
// no grid-wide synchronisation is needed.
#include "kernels.h"

#include <type_traits>

namespace psms {

struct BlockArgs {
  Geo g;
  const void* links[MAXPROP];
  void* rho;
  void* x;
  void* delta;
  void* pbuf;
  size_t rhs_stride;  // units
  int nrhs, colour, niter;
  double tol, kappa;
  int face;  // 1: first apply the residual update across the block faces (see face_update)
  int lanes;  // LDS-resident form: 1 or 2 lanes per site (0: by grid size)
  int eo;     // 1: even-odd preconditioned minimal residual (k_block_mr_eo, k_block_mr_eo_g);
              // 2: the same with 12-real links read from L2 instead of LDS
  const void* rho_in;  // non-null: read the initial rho from here (same shape) instead of rho
  int x_assign;        // 1: x = delta instead of x += delta (x need not be initialised)
  int eo_lanes;        // even-odd form on 256-site FP32 blocks: lanes per site (2, 4; 0 = by grid)
  int xcd_map;         // 1: workgroup order by XCD (block_coord)
  int rin_f32;         // 1: rho_in is an FP32 field (units of rin_stride per right-hand side)
  int link16;          // Schwarz sweeps of the two-lane even-odd form: 1 staged 12-real links in
                       // FP16; 2 whole FP16 links and FP16 exchange fields
  size_t rin_stride;
  int* iters;
};

// Workgroup -> (block, right-hand side, proposal). The grid is (blocks of the colour,
// right-hand sides, proposals), and workgroups are dealt to the 8 XCDs in turn, in the
// order of their linear index w. With xcd_map, w is read as XCD w % 8 and position
// w / 8 on it: consecutive positions on one XCD are the right-hand sides of one block,
// which hop over the same links, so those reads meet in that XCD's L2; each XCD takes
// a contiguous range of (proposal, block) pairs, whose faces neighbour each other.
struct BlockCoord {
  int blk, rhs, prop;
};
__device__ __forceinline__ BlockCoord block_coord(const BlockArgs& a) {
  const int nb = gridDim.x, nr = gridDim.y, np = gridDim.z;
  if (a.xcd_map && ((nb * np) & 7) == 0) {
    const int w = blockIdx.x + nb * (blockIdx.y + nr * blockIdx.z);
    const int i = w >> 3;
    const int q = (w & 7) * ((nb * np) >> 3) + i / nr;
    return {a.colour * a.g.nblk_c + q % nb, i % nr, q / nb};
  }
  return {a.colour * a.g.nblk_c + int(blockIdx.x), int(blockIdx.y), int(blockIdx.z)};
}

// The initial residual of parity par at site s of right-hand side rix (proposal-major
// index): from rho (already offset to that right-hand side), or from rho_in, which has the
// kernel's storage or, with rin_f32, FP32 (the first Schwarz sweep reading an FP32 Krylov
// residual directly, with no converted copy).
template <class S, class T>
__device__ __forceinline__ void load_rho0(const BlockArgs& a, const typename S::unit* rho, size_t rix, int par, int s,
                                          Spinor<T>& v) {
  const size_t Vh = a.g.Vh;
  if (a.rho_in && a.rin_f32) {
    StF32::load(reinterpret_cast<const float4*>(a.rho_in) + rix * a.rin_stride + size_t(par) * StF32::NC * Vh, Vh, s, v);
  } else {
    const typename S::unit* base = a.rho_in ? reinterpret_cast<const typename S::unit*>(a.rho_in) + rix * a.rhs_stride : rho;
    S::load(base + size_t(par) * S::NC * Vh, Vh, s, v);
  }
}

// Schwarz residual update across the faces of a block of colour c:
// rho_c -= D_{c,c'} delta_c', i.e. acc += kappa * (the hops of site (p, s) that
// leave its block, applied to delta of the neighbouring blocks, which all have the
// other colour c' and hold the deltas of that colour's last sweep). Only sites of
// the other colour are read, so the blocks of colour c can update in parallel.
template <class S, class LK, class T>
__device__ __forceinline__ void face_update(const Geo& g, const typename LK::unit* __restrict__ lk,
                                            const typename S::unit* __restrict__ dl, int p, int s, T kp, Spinor<T>& acc) {
  const size_t Vh = g.Vh;
  SiteInfo si;
  site_info(g, p, s, si);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Nbr n = neighbour(g, si, mu, +1);
    if (n.cross) {
      SU3<T> U;
      LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
      Spinor<T> nb;
      S::load(dl + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_fwd(mu, U, nb, kp * T(n.sign), acc);
    }
    n = neighbour(g, si, mu, -1);
    if (n.cross) {
      SU3<T> U;
      LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
      Spinor<T> nb;
      S::load(dl + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_bwd(mu, U, nb, kp * T(n.sign), acc);
    }
  }
}

// (D_b r)(x) for one site: r(x) - kappa * sum of the intra-block hops.
template <class S, class LK, class T>
__device__ __forceinline__ void block_op_site(const Geo& g, const typename LK::unit* __restrict__ lk,
                                              const typename S::unit* __restrict__ r, int p, int s, T mk, Spinor<T>& out) {
  const size_t Vh = g.Vh;
  SiteInfo si;
  site_info(g, p, s, si);
  zero(out);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Nbr n = neighbour(g, si, mu, +1);
    if (!n.cross) {
      SU3<T> U;
      LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
      Spinor<T> nb;
      S::load(r + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_fwd(mu, U, nb, mk, out);
    }
    n = neighbour(g, si, mu, -1);
    if (!n.cross) {
      SU3<T> U;
      LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
      Spinor<T> nb;
      S::load(r + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_bwd(mu, U, nb, mk, out);
    }
  }
  Spinor<T> d;
  S::load(r + size_t(p) * S::NC * Vh, Vh, s, d);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) out.v[a][c] = out.v[a][c] + d.v[a][c];
}

__device__ __forceinline__ double wg_sum(double v, double* sm) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sm[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) t += sm[k];
  return t;
}

// Three workgroup sums with one barrier pair (fixed order, deterministic).
__device__ __forceinline__ void wg_sum3(double& a, double& b, double& c, double (*sm)[16]) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sm[0][w] = a;
    sm[1][w] = b;
    sm[2][w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) {
    a += sm[0][k];
    b += sm[1][k];
    c += sm[2][k];
  }
}

template <class S, class LK, class T>
__global__ void __launch_bounds__(256) k_block_mr(BlockArgs a) {
  __shared__ double sm3[3][16];
  double* sm = sm3[0];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  unit* pb = reinterpret_cast<unit*>(a.pbuf) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const int nsite = 2 * g.Vbh;
  const T mk = T(-a.kappa);

  // rho_b += face update (optional), delta = 0, |rho_b|^2
  double b2 = 0.0;
  for (int j = threadIdx.x; j < nsite; j += blockDim.x) {
    int p = j / g.Vbh, s = blk * g.Vbh + (j - p * g.Vbh);
    Spinor<T> v, z;
    load_rho0<S>(a, rho, rix, p, s, v);
    if (a.face) face_update<S, LK, T>(g, lk, dl, p, s, T(a.kappa), v);
    if (a.face || a.rho_in) S::store(rho + size_t(p) * S::NC * Vh, Vh, s, v);
    zero(z);
    S::store(dl + size_t(p) * S::NC * Vh, Vh, s, z);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) b2 += double(v.v[q][c].re) * v.v[q][c].re + double(v.v[q][c].im) * v.v[q][c].im;
  }
  b2 = wg_sum(b2, sm);
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 : -1.0;

  int it = 0;
  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
      // p = D_b r,  (p, r) and |p|^2
      double prr = 0.0, pri = 0.0, pp = 0.0;
      for (int j = threadIdx.x; j < nsite; j += blockDim.x) {
        int p = j / g.Vbh, s = blk * g.Vbh + (j - p * g.Vbh);
        Spinor<T> Dr, r;
        block_op_site<S, LK, T>(g, lk, rho, p, s, mk, Dr);
        S::load(rho + size_t(p) * S::NC * Vh, Vh, s, r);
        S::store(pb + size_t(p) * S::NC * Vh, Vh, s, Dr);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double ar = Dr.v[q][c].re, ai = Dr.v[q][c].im, br = r.v[q][c].re, bi = r.v[q][c].im;
            prr += ar * br + ai * bi;
            pri += ar * bi - ai * br;
            pp += ar * ar + ai * ai;
          }
      }
      wg_sum3(prr, pri, pp, sm3);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
      for (int j = threadIdx.x; j < nsite; j += blockDim.x) {
        int p = j / g.Vbh, s = blk * g.Vbh + (j - p * g.Vbh);
        Spinor<T> r, pv, d;
        S::load(rho + size_t(p) * S::NC * Vh, Vh, s, r);
        S::load(pb + size_t(p) * S::NC * Vh, Vh, s, pv);
        S::load(dl + size_t(p) * S::NC * Vh, Vh, s, d);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
            r.v[q][c] = r.v[q][c] - cmul(alpha, pv.v[q][c]);
            rr += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
          }
        S::store(dl + size_t(p) * S::NC * Vh, Vh, s, d);
        S::store(rho + size_t(p) * S::NC * Vh, Vh, s, r);
      }
      rr = wg_sum(rr, sm);  // also orders the rho stores before the next sweep reads them
      if (rr <= stop2) { ++it; break; }
    }
  }
  // x += delta
  for (int j = threadIdx.x; j < nsite; j += blockDim.x) {
    int p = j / g.Vbh, s = blk * g.Vbh + (j - p * g.Vbh);
    Spinor<T> d, xv;
    S::load(dl + size_t(p) * S::NC * Vh, Vh, s, d);
    if (a.x_assign) zero(xv);
    else S::load(x + size_t(p) * S::NC * Vh, Vh, s, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
    S::store(x + size_t(p) * S::NC * Vh, Vh, s, xv);
  }
  if (a.iters && threadIdx.x == 0) atomicMax(a.iters, it);
}

// acc += c * (the intra-block hops of site (p, s), applied to src on the other parity)
template <class S, class LK, class T>
__device__ __forceinline__ void block_half_hops(const Geo& g, const typename LK::unit* __restrict__ lk,
                                                const typename S::unit* __restrict__ src, int p, int s, T c,
                                                Spinor<T>& acc) {
  const size_t Vh = g.Vh;
  SiteInfo si;
  site_info(g, p, s, si);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Nbr n = neighbour(g, si, mu, +1);
    if (!n.cross) {
      SU3<T> U;
      LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
      Spinor<T> nb;
      S::load(src + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_fwd(mu, U, nb, c, acc);
    }
    n = neighbour(g, si, mu, -1);
    if (!n.cross) {
      SU3<T> U;
      LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
      Spinor<T> nb;
      S::load(src + size_t(1 - p) * S::NC * Vh, Vh, n.s, nb);
      hop_bwd(mu, U, nb, c, acc);
    }
  }
}

// Even-odd form of the global-memory block solver (any block size): minimal residual
// on each block's even Schur complement 1 - k^2 H_eo H_oe (as in k_block_mr_eo), with
// the fields in global memory. Per iteration the odd sites form t = k H_oe r (odd half
// of pbuf), the even sites p = r - k H_eo t (even half) with the three inner products,
// then the even sites update. rho's even half holds the residual, delta's even half
// the iterate; at the end delta_o = rho_o + k H_oe delta_e and the odd residual is zero.
// Per iteration this moves about the data of one plain iteration and reduces the
// residual about as much as two.
template <class S, class LK, class T>
__global__ void __launch_bounds__(256) k_block_mr_eo_g(BlockArgs a) {
  __shared__ double sm[3][16];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  unit* pb = reinterpret_cast<unit*>(a.pbuf) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const int H = g.Vbh;
  const T kp = T(a.kappa), mk = T(-a.kappa);
  const size_t odd = size_t(S::NC) * Vh;  // offset of the odd half of a field

  // rho_b += face update (optional), |rho_b|^2
  double b2 = 0.0;
  for (int j = threadIdx.x; j < 2 * H; j += blockDim.x) {
    const int p = j / H, s = blk * H + (j - p * H);
    Spinor<T> v;
    load_rho0<S>(a, rho, rix, p, s, v);
    if (a.face) face_update<S, LK, T>(g, lk, dl, p, s, kp, v);
    if (a.face || a.rho_in) S::store(rho + p * odd, Vh, s, v);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) b2 += double(v.v[q][c].re) * v.v[q][c].re + double(v.v[q][c].im) * v.v[q][c].im;
  }
  b2 = wg_sum(b2, sm[0]);  // also orders the rho stores before the next pass reads them
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 : -1.0;
  // even right-hand side rho_e + k H_eo rho_o (into rho_e), delta_e = 0
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    const int s = blk * H + j;
    Spinor<T> v, z;
    S::load(rho, Vh, s, v);
    block_half_hops<S, LK, T>(g, lk, rho, 0, s, kp, v);
    S::store(rho, Vh, s, v);
    zero(z);
    S::store(dl, Vh, s, z);
  }
  __syncthreads();

  int it = 0;
  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
      // t = k H_oe r on the odd sites
      for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const int s = blk * H + j;
        Spinor<T> t;
        zero(t);
        block_half_hops<S, LK, T>(g, lk, rho, 1, s, kp, t);
        S::store(pb + odd, Vh, s, t);
      }
      __syncthreads();
      // p = r - k H_eo t on the even sites, (p, r) and |p|^2
      double prr = 0.0, pri = 0.0, pp = 0.0;
      for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const int s = blk * H + j;
        Spinor<T> r, pv;
        S::load(rho, Vh, s, r);
        pv = r;
        block_half_hops<S, LK, T>(g, lk, pb, 0, s, mk, pv);
        S::store(pb, Vh, s, pv);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double ar = pv.v[q][c].re, ai = pv.v[q][c].im, br = r.v[q][c].re, bi = r.v[q][c].im;
            prr += ar * br + ai * bi;
            pri += ar * bi - ai * br;
            pp += ar * ar + ai * ai;
          }
      }
      wg_sum3(prr, pri, pp, sm);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
      for (int j = threadIdx.x; j < H; j += blockDim.x) {
        const int s = blk * H + j;
        Spinor<T> r, pv, d;
        S::load(rho, Vh, s, r);
        S::load(pb, Vh, s, pv);
        S::load(dl, Vh, s, d);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
            r.v[q][c] = r.v[q][c] - cmul(alpha, pv.v[q][c]);
            rr += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
          }
        S::store(dl, Vh, s, d);
        S::store(rho, Vh, s, r);
      }
      rr = wg_sum(rr, sm[0]);  // also orders the rho_e stores before the next pass reads them
      if (rr <= stop2) {
        ++it;
        break;
      }
    }
  }
  __syncthreads();
  // delta_o = rho_o + k H_oe delta_e, rho_o = 0; x += delta on both parities
  for (int j = threadIdx.x; j < H; j += blockDim.x) {
    const int s = blk * H + j;
    Spinor<T> d, z, xv;
    S::load(rho + odd, Vh, s, d);
    block_half_hops<S, LK, T>(g, lk, dl, 1, s, kp, d);
    S::store(dl + odd, Vh, s, d);
    zero(z);
    S::store(rho + odd, Vh, s, z);
    if (a.x_assign) zero(xv);
    else S::load(x + odd, Vh, s, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
    S::store(x + odd, Vh, s, xv);
    S::load(dl, Vh, s, d);
    if (a.x_assign) zero(xv);
    else S::load(x, Vh, s, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
    S::store(x, Vh, s, xv);
  }
  if (a.iters && threadIdx.x == 0) atomicMax(a.iters, it);
}

// LDS-resident variant for blocks of VB sites (one thread per site, VB <= 256).
// The block's forward links are staged once in LDS (12-real links as float4
// planes, or FP64 links left in global memory / L2 when LK is LkF64); the
// residual lives in registers and is exchanged through LDS for the hops. Each
// MR iteration touches no global memory.
template <class LK> struct LdsLinks {
  static constexpr bool on = false;
};
template <> struct LdsLinks<LkF32C12> {
  static constexpr bool on = true;
};

template <class S, class LK, class T, int VB>
__global__ void __launch_bounds__(VB) k_block_mr_lds(BlockArgs a) {
  constexpr bool LL = LdsLinks<LK>::on;
  __shared__ cx<T> r_lds[12][VB];
  __shared__ float4 lk_lds[LL ? 4 * 3 : 1][LL ? VB : 1];
  __shared__ double sm[3][16];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const T mk = T(-a.kappa);
  const int t = threadIdx.x;
  const int Vbh = VB / 2;
  const int p = t < Vbh ? 0 : 1;
  const int s = blk * Vbh + (t - p * Vbh);

  // neighbour thread of each hop inside the block (-1: leaves the block)
  int nbt[8];
  int nbs[8];
  {
    SiteInfo si;
    site_info(g, p, s, si);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        Nbr n = neighbour(g, si, mu, d == 0 ? +1 : -1);
        nbs[2 * mu + d] = n.s;
        nbt[2 * mu + d] = n.cross ? -1 : (1 - p) * Vbh + (n.s - blk * Vbh);
      }
    }
  }
  if constexpr (LL) {
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int k = 0; k < 3; ++k) lk_lds[mu * 3 + k][t] = reinterpret_cast<const float4*>(lk)[(size_t(p * 4 + mu) * 3 + k) * Vh + s];
  }
  Spinor<T> r, d;
  load_rho0<S>(a, rho, rix, p, s, r);
  if (a.face) face_update<S, LK, T>(g, lk, dl, p, s, T(a.kappa), r);
  zero(d);
  double b2 = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) b2 += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
  b2 = wg_sum(b2, sm[0]);
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 : -1.0;

  int it = 0;
  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
#pragma unroll
      for (int k = 0; k < 12; ++k) r_lds[k][t] = r.v[k / 3][k % 3];
      __syncthreads();
      Spinor<T> pv = r;
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
        for (int dd = 0; dd < 2; ++dd) {
          const int tn = nbt[2 * mu + dd];
          if (tn >= 0) {
            SU3<T> U;
            const int lt = dd == 0 ? t : tn;  // forward hop: own link; backward: neighbour's
            if constexpr (LL) {
#pragma unroll
              for (int k = 0; k < 3; ++k) {
                float4 v = lk_lds[mu * 3 + k][lt];
                U.m[(2 * k) / 3][(2 * k) % 3] = {T(v.x), T(v.y)};
                U.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(v.z), T(v.w)};
              }
              su3_row2(U, T(1));
            } else {
              const int lp = dd == 0 ? p : 1 - p;
              const int ls = dd == 0 ? s : nbs[2 * mu + dd];
              LK::load(lk + size_t(lp * 4 + mu) * LK::NC * Vh, Vh, ls, U);
            }
            Spinor<T> nb;
#pragma unroll
            for (int k = 0; k < 12; ++k) nb.v[k / 3][k % 3] = r_lds[k][tn];
            if (dd == 0) hop_fwd(mu, U, nb, mk, pv);
            else hop_bwd(mu, U, nb, mk, pv);
          }
        }
      }
      double prr = 0.0, pri = 0.0, pp = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double ar = pv.v[q][c].re, ai = pv.v[q][c].im, br = r.v[q][c].re, bi = r.v[q][c].im;
          prr += ar * br + ai * bi;
          pri += ar * bi - ai * br;
          pp += ar * ar + ai * ai;
        }
      wg_sum3(prr, pri, pp, sm);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
          r.v[q][c] = r.v[q][c] - cmul(alpha, pv.v[q][c]);
          rr += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
        }
      if (stop2 > 0) {
        rr = wg_sum(rr, sm[0]);
        if (rr <= stop2) {
          ++it;
          break;
        }
      }
    }
  }
  S::store(rho + size_t(p) * S::NC * Vh, Vh, s, r);
  S::store(dl + size_t(p) * S::NC * Vh, Vh, s, d);
  Spinor<T> xv;
  if (a.x_assign) zero(xv);
  else S::load(x + size_t(p) * S::NC * Vh, Vh, s, xv);
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
  S::store(x + size_t(p) * S::NC * Vh, Vh, s, xv);
  if (a.iters && t == 0) atomicMax(a.iters, it);
}


// Two lanes per site (512 threads, LDS-resident links for 12-real link storage):
// waves 0-3 take the forward hops, the MR update and the residual of their site;
// waves 4-7 take the backward hops and hand their partial sum over through LDS.
// Twice the waves per block hide the LDS and barrier latency of a block solve
// whose grid is too small to give every SIMD more than one wave.
template <class S, class LK, class T>
__global__ void __launch_bounds__(512) k_block_mr_lds2(BlockArgs a) {
  constexpr int VB = 256;
  static_assert(LdsLinks<LK>::on, "two-lane form stages 12-real links in LDS");
  __shared__ cx<T> r_lds[12][VB];
  __shared__ cx<T> q_lds[12][VB];
  __shared__ float4 lk_lds[4 * 3][VB];
  __shared__ double sm[3][16];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const T mk = T(-a.kappa);
  const int t = threadIdx.x & (VB - 1);
  const int h = threadIdx.x >> 8;  // wave-uniform: 0 forward hops, 1 backward hops
  const int Vbh = VB / 2;
  const int p = t < Vbh ? 0 : 1;
  const int s = blk * Vbh + (t - p * Vbh);

  int nbt[4];  // neighbour thread of this lane's four hops (-1: leaves the block)
  {
    SiteInfo si;
    site_info(g, p, s, si);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      Nbr n = neighbour(g, si, mu, h == 0 ? +1 : -1);
      nbt[mu] = n.cross ? -1 : (1 - p) * Vbh + (n.s - blk * Vbh);
    }
  }
  // each half stages the link planes of two directions
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int mu = 2 * h + k / 3, kk = k % 3;
    lk_lds[mu * 3 + kk][t] = reinterpret_cast<const float4*>(lk)[(size_t(p * 4 + mu) * 3 + kk) * Vh + s];
  }
  Spinor<T> r, d;
  zero(r);
  zero(d);
  double b2 = 0.0;
  if (h == 0) {
    load_rho0<S>(a, rho, rix, p, s, r);
    if (a.face) face_update<S, LK, T>(g, lk, dl, p, s, T(a.kappa), r);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) b2 += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
  }
  b2 = wg_sum(b2, sm[0]);
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 : -1.0;

  int it = 0;
  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
      if (h == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) r_lds[k][t] = r.v[k / 3][k % 3];
      }
      __syncthreads();
      Spinor<T> acc;
      if (h == 0) acc = r;
      else zero(acc);
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        const int tn = nbt[mu];
        if (tn >= 0) {
          SU3<T> U;
          const int lt = h == 0 ? t : tn;  // forward hop: own link; backward: the neighbour's
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            float4 v = lk_lds[mu * 3 + k][lt];
            U.m[(2 * k) / 3][(2 * k) % 3] = {T(v.x), T(v.y)};
            U.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(v.z), T(v.w)};
          }
          su3_row2(U, T(1));
          Spinor<T> nb;
#pragma unroll
          for (int k = 0; k < 12; ++k) nb.v[k / 3][k % 3] = r_lds[k][tn];
          if (h == 0) hop_fwd(mu, U, nb, mk, acc);
          else hop_bwd(mu, U, nb, mk, acc);
        }
      }
      if (h == 1) {
#pragma unroll
        for (int k = 0; k < 12; ++k) q_lds[k][t] = acc.v[k / 3][k % 3];
      }
      __syncthreads();
      double prr = 0.0, pri = 0.0, pp = 0.0;
      if (h == 0) {
#pragma unroll
        for (int k = 0; k < 12; ++k) acc.v[k / 3][k % 3] = acc.v[k / 3][k % 3] + q_lds[k][t];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double ar = acc.v[q][c].re, ai = acc.v[q][c].im, br = r.v[q][c].re, bi = r.v[q][c].im;
            prr += ar * br + ai * bi;
            pri += ar * bi - ai * br;
            pp += ar * ar + ai * ai;
          }
      }
      wg_sum3(prr, pri, pp, sm);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
      if (h == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
            r.v[q][c] = r.v[q][c] - cmul(alpha, acc.v[q][c]);
            rr += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
          }
      }
      if (stop2 > 0) {
        rr = wg_sum(rr, sm[0]);
        if (rr <= stop2) {
          ++it;
          break;
        }
      }
    }
  }
  if (h == 0) {
    S::store(rho + size_t(p) * S::NC * Vh, Vh, s, r);
    S::store(dl + size_t(p) * S::NC * Vh, Vh, s, d);
    Spinor<T> xv;
    if (a.x_assign) zero(xv);
    else S::load(x + size_t(p) * S::NC * Vh, Vh, s, xv);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
    S::store(x + size_t(p) * S::NC * Vh, Vh, s, xv);
    if (a.iters && t == 0) atomicMax(a.iters, it);
  }
}


// Even-odd preconditioned block solver for 256-site blocks (256 threads). With e/o
// the two parities of the block, D_b = [[1, -k H_eo], [-k H_oe, 1]] and
//   D_b x = rho  <=>  (1 - k^2 H_eo H_oe) x_e = rho_e + k H_eo rho_o,  x_o = rho_o + k H_oe x_e.
// Minimal residual runs on the even Schur complement, whose spectral radius around 1
// is about the square of that of D_b, so an iteration reduces the residual about as
// much as two iterations on D_b. Afterwards the block residual rho - D_b delta is the
// minimal-residual residual on the even sites and exactly zero on the odd sites.
// Thread (j, h): site j of each parity; every hop phase gives each site two lanes
// (h = 0 forward hops, h = 1 backward hops, wave-uniform), so no SIMD idles while
// only one parity computes. The even-site state lives in lane 0, the odd in lane 1.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));

// FP16 arithmetic of the Schwarz sweeps: a spinor as 12 and an SU(3) matrix as 9 packed
// (re, im) pairs. Spin projections, colour products and hop sums run on the pairs with
// packed FP16 instructions (a complex multiply-add is two packed FMAs, the broadcasts and
// swaps being operand modifiers); the iterate and residual stay in FP32.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
struct SpinorH { h2_t v[4][3]; };
struct SU3H { h2_t m[3][3]; };
__device__ __forceinline__ h2_t h_ti(h2_t a) { return h2_t{-a.y, a.x}; }
__device__ __forceinline__ h2_t h_tmi(h2_t a) { return h2_t{a.y, -a.x}; }
__device__ __forceinline__ h2_t h_fma(h2_t a, h2_t b, h2_t c) { return __builtin_elementwise_fma(a, b, c); }
__device__ __forceinline__ uint32_t h_pack(cx<float> z) {
  return __builtin_bit_cast(uint32_t, h2_t{_Float16(z.re), _Float16(z.im)});
}
__device__ __forceinline__ cx<float> h_unpack(uint32_t w) {
  const h2_t z = __builtin_bit_cast(h2_t, w);
  return {float(z.x), float(z.y)};
}
__device__ __forceinline__ cx<float> h_f32(h2_t z) { return {float(z.x), float(z.y)}; }
// o = U v: u v = u.re (v.re, v.im) + u.im (-v.im, v.re)
__device__ __forceinline__ void su3h_mul(const SU3H& u, const h2_t (&v)[3], h2_t (&o)[3]) {
  h2_t vs[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) vs[b] = h2_t{-v[b].y, v[b].x};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h2_t c = u.m[a][0].xx * v[0];
    c = h_fma(u.m[a][0].yy, vs[0], c);
    c = h_fma(u.m[a][1].xx, v[1], c);
    c = h_fma(u.m[a][1].yy, vs[1], c);
    c = h_fma(u.m[a][2].xx, v[2], c);
    o[a] = h_fma(u.m[a][2].yy, vs[2], c);
  }
}
// o = U^+ v: conj(u) v = u.re (v.re, v.im) + u.im (v.im, -v.re)
__device__ __forceinline__ void su3h_dag_mul(const SU3H& u, const h2_t (&v)[3], h2_t (&o)[3]) {
  h2_t vs[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) vs[b] = h2_t{v[b].y, -v[b].x};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h2_t c = u.m[0][a].xx * v[0];
    c = h_fma(u.m[0][a].yy, vs[0], c);
    c = h_fma(u.m[1][a].xx, v[1], c);
    c = h_fma(u.m[1][a].yy, vs[1], c);
    c = h_fma(u.m[2][a].xx, v[2], c);
    o[a] = h_fma(u.m[2][a].yy, vs[2], c);
  }
}
template <int SG> __device__ __forceinline__ void h_acc(h2_t& a, h2_t x) { a = SG > 0 ? a + x : a - x; }
// acc += SG U(x,mu) (1 - gamma_mu) psi(x+mu) and acc += SG U(x-mu,mu)^+ (1 + gamma_mu) psi(x-mu):
// the projections and reconstructions of hop_fwd and hop_bwd (chiral basis) on FP16 pairs
template <int SG> __device__ __forceinline__ void hoph_fwd(int mu, const SU3H& U, const SpinorH& p, SpinorH& acc) {
  h2_t h0[3], h1[3], u0[3], u1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    switch (mu) {
      case 0: h0[a] = p.v[0][a] + p.v[2][a]; h1[a] = p.v[1][a] + p.v[3][a]; break;
      case 1: h0[a] = p.v[0][a] + h_ti(p.v[3][a]); h1[a] = p.v[1][a] + h_ti(p.v[2][a]); break;
      case 2: h0[a] = p.v[0][a] + p.v[3][a]; h1[a] = p.v[1][a] - p.v[2][a]; break;
      default: h0[a] = p.v[0][a] + h_ti(p.v[2][a]); h1[a] = p.v[1][a] - h_ti(p.v[3][a]); break;
    }
  }
  su3h_mul(U, h0, u0);
  su3h_mul(U, h1, u1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h_acc<SG>(acc.v[0][a], u0[a]);
    h_acc<SG>(acc.v[1][a], u1[a]);
    switch (mu) {
      case 0: h_acc<SG>(acc.v[2][a], u0[a]); h_acc<SG>(acc.v[3][a], u1[a]); break;
      case 1: h_acc<SG>(acc.v[2][a], h_tmi(u1[a])); h_acc<SG>(acc.v[3][a], h_tmi(u0[a])); break;
      case 2: h_acc<-SG>(acc.v[2][a], u1[a]); h_acc<SG>(acc.v[3][a], u0[a]); break;
      default: h_acc<SG>(acc.v[2][a], h_tmi(u0[a])); h_acc<SG>(acc.v[3][a], h_ti(u1[a])); break;
    }
  }
}
template <int SG> __device__ __forceinline__ void hoph_bwd(int mu, const SU3H& U, const SpinorH& p, SpinorH& acc) {
  h2_t h0[3], h1[3], w0[3], w1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    switch (mu) {
      case 0: h0[a] = p.v[0][a] - p.v[2][a]; h1[a] = p.v[1][a] - p.v[3][a]; break;
      case 1: h0[a] = p.v[0][a] + h_tmi(p.v[3][a]); h1[a] = p.v[1][a] + h_tmi(p.v[2][a]); break;
      case 2: h0[a] = p.v[0][a] - p.v[3][a]; h1[a] = p.v[1][a] + p.v[2][a]; break;
      default: h0[a] = p.v[0][a] + h_tmi(p.v[2][a]); h1[a] = p.v[1][a] + h_ti(p.v[3][a]); break;
    }
  }
  su3h_dag_mul(U, h0, w0);
  su3h_dag_mul(U, h1, w1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    h_acc<SG>(acc.v[0][a], w0[a]);
    h_acc<SG>(acc.v[1][a], w1[a]);
    switch (mu) {
      case 0: h_acc<-SG>(acc.v[2][a], w0[a]); h_acc<-SG>(acc.v[3][a], w1[a]); break;
      case 1: h_acc<SG>(acc.v[2][a], h_ti(w1[a])); h_acc<SG>(acc.v[3][a], h_ti(w0[a])); break;
      case 2: h_acc<SG>(acc.v[2][a], w1[a]); h_acc<-SG>(acc.v[3][a], w0[a]); break;
      default: h_acc<SG>(acc.v[2][a], h_ti(w0[a])); h_acc<-SG>(acc.v[3][a], h_ti(w1[a])); break;
    }
  }
}

template <class S, class LK, class T, bool STAGE = true, int L16 = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(L16 ? 3 : 1))) k_block_mr_eo(BlockArgs a) {
  constexpr int H = 128;  // sites per parity
  // STAGE: 12-real links staged in LDS times kappa (73 KB in FP32, two workgroups per CU),
  // so that a hop neither scales its result nor multiplies by kappa; otherwise read from L2
  // at each hop (24 KB). For Schwarz sweeps, whose fixed iteration counts do not need the
  // last bits of the operator, L16 = 1 stages the 12-real links in FP16 (49 KB, three
  // workgroups per CU), and L16 = 2 stages whole links in FP16 and exchanges the fields
  // between lanes in FP16 too (49 KB): each hop then reads 84 bytes of LDS instead of 120,
  // rebuilds no row and converts nothing. The FP16 fields are the block's own, scaled to
  // unit RMS per component (the minimal-residual iteration is homogeneous; its
  // coefficients do not change), so their range is that of FP16 at any residual size.
  constexpr bool LL = LdsLinks<LK>::on && STAGE;
  constexpr bool LH = LL && L16 == 1;
  constexpr bool XH = LL && L16 == 2 && sizeof(T) == 4;
  constexpr int NE = XH ? 1 : 12, NH = XH ? 1 : H;
  __shared__ cx<T> ev[NE][NH];  // an even-site field; after a hop phase, lane 1's even partial sum
  __shared__ cx<T> od[NE][NH];  // an odd-site field (the two lanes' hop sums, added in turn)
  __shared__ float4 lk_lds[LL && !LH && !XH ? 12 : 1][LL && !LH && !XH ? 2 * H : 1];
  __shared__ uint2 lk_h[LH ? 12 : 1][LH ? 2 * H : 1];
  // FP16 form (48 KB): the two fields in FP16 (four pairs per unit), then the whole FP16
  // links, link (gp, mu, q) at index (gp * 4 + mu) * H + q in pairs 0-3, 4-7 and 8. Before
  // the links are staged, the same memory holds the face hops of 4^4 blocks in FP32.
  __shared__ uint4 xlds[XH ? 24 * H : 1];
  uint4(*evh)[H] = reinterpret_cast<uint4(*)[H]>(xlds);
  uint4(*odh)[H] = reinterpret_cast<uint4(*)[H]>(xlds + 3 * H);
  uint4* lk_a = xlds + 6 * H;
  uint4* lk_b = xlds + 14 * H;
  uint32_t* lk_c = reinterpret_cast<uint32_t*>(xlds + 22 * H);
  float4(*fc)[4 * H] = reinterpret_cast<float4(*)[4 * H]>(xlds);  // [6][512]: face hop t, 12 complex
  __shared__ double sm[3][16];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const T kp = T(a.kappa);
  const int j = threadIdx.x & (H - 1);
  const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);
  const int s = blk * H + j;  // index of site j in either parity array

  // in-block neighbours of this lane's four hops: nA for the odd site j (even
  // neighbours), nB for the even site j (odd neighbours); -1 when the hop leaves the block
  int nA[4], nB[4], gA[4], gB[4], lo[4];
  if constexpr (XH) {
    // in-block neighbours from the local coordinates alone: x + dir mu stays in the block
    // when 0 <= l_mu + dir < b_mu, at in-block index (locallex + dir sl_mu) / 2
    const uint32_t w1 = g.lcoord[g.Vbh + j], w0 = g.lcoord[j];
    int l1[4], l0[4], x1 = 0, x0 = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      l1[m] = (w1 >> (8 * m)) & 255;
      l0[m] = (w0 >> (8 * m)) & 255;
      x1 += l1[m] * g.sl[m];
      x0 += l0[m] * g.sl[m];
    }
    const int dir = h == 0 ? 1 : -1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int t1 = l1[mu] + dir, t0 = l0[mu] + dir;
      nA[mu] = (t1 >= 0 && t1 < g.b[mu]) ? (x1 + dir * g.sl[mu]) >> 1 : -1;
      nB[mu] = (t0 >= 0 && t0 < g.b[mu]) ? (x0 + dir * g.sl[mu]) >> 1 : -1;
      gA[mu] = gB[mu] = 0;  // the L2-link path only
      lo[mu] = h ? l1[mu] : l0[mu];
    }
  } else {
    SiteInfo so, se;
    site_info(g, 1, s, so);
    site_info(g, 0, s, se);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      Nbr n = neighbour(g, so, mu, h == 0 ? +1 : -1);
      nA[mu] = n.cross ? -1 : n.s - blk * H;
      gA[mu] = n.s;
      Nbr m = neighbour(g, se, mu, h == 0 ? +1 : -1);
      nB[mu] = m.cross ? -1 : m.s - blk * H;
      gB[mu] = m.s;
      lo[mu] = h ? so.l[mu] : se.l[mu];  // local coordinates of this lane's own site
    }
  }
  const float kf = float(a.kappa), ik = float(1.0 / a.kappa);
  if constexpr (LL && !XH) {  // lane h stages kappa times the forward links of site j of parity h
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      float4 v = reinterpret_cast<const float4*>(lk)[(size_t(h * 4 + k / 3) * 3 + k % 3) * Vh + s];
      if constexpr (LH) {
        const half4_t hv = {_Float16(kf * v.x), _Float16(kf * v.y), _Float16(kf * v.z), _Float16(kf * v.w)};
        lk_h[k][h * H + j] = __builtin_bit_cast(uint2, hv);
      } else {
        lk_lds[k][h * H + j] = make_float4(kf * v.x, kf * v.y, kf * v.z, kf * v.w);
      }
    }
  }
  // own site (parity h): rho (+ the face update)
  Spinor<T> r, d, acc;
  load_rho0<S>(a, rho, rix, h, s, r);
  // FP16 form: the links to stage are written after the face update, whose hops use the
  // same LDS; they are fetched as soon as the face hops are done, so that their latency
  // overlaps the gather
  float4 lraw[XH ? 12 : 1];
  auto fetch_links = [&]() {
    static_assert(!XH || std::is_same<LK, LkF32C12>::value, "the FP16 form stages 12-real FP32 links");
#pragma unroll
    for (int k = 0; k < 12; ++k) lraw[k] = reinterpret_cast<const float4*>(lk)[(size_t(h * 4 + k / 3) * 3 + k % 3) * Vh + s];
  };
  if constexpr (XH) {
    // Face update of a 4^4 block: the 512 hops that enter it from its eight neighbours,
    // two per lane and every lane busy. Hop t runs in direction t >> 7, forward from the
    // face l_mu = 3 when t & 64 is 0, else backward from the face l_mu = 0; t & 63 holds
    // the other three local coordinates, two bits each in increasing direction order. The
    // hops go to LDS in FP32 and each lane adds those of its own site, in direction order.
    if (a.face && g.b[0] == 4 && g.b[1] == 4 && g.b[2] == 4 && g.b[3] == 4) {
      SiteInfo si;
      const uint32_t bw = g.bcoord[blk];
#pragma unroll
      for (int m = 0; m < 4; ++m) si.B[m] = (bw >> (8 * m)) & 255;
      si.colour = blk >= g.nblk_c ? 1 : 0;
      si.lexB = 2 * (blk - si.colour * g.nblk_c) + (si.B[3] & 1);
      // hop t in direction MU (a constant, so that the site tables index statically)
      auto face_hop = [&](auto MU, int t) {
        constexpr int mu = decltype(MU)::value;
        const bool fwd = __builtin_amdgcn_readfirstlane((t >> 6) & 1) == 0;
        int ll = 0, par = 0, c = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          int l;
          if (m == mu) {
            l = fwd ? 3 : 0;
          } else {
            l = (t >> (2 * c)) & 3;
            ++c;
          }
          si.l[m] = l;
          ll += l * g.sl[m];
          par += l;
        }
        par &= 1;
        si.locallex = ll;
        const Nbr n = neighbour(g, si, mu, fwd ? +1 : -1);
        Spinor<T> nb, f;
        zero(f);
        S::load(dl + size_t(1 - par) * S::NC * Vh, Vh, n.s, nb);
        SU3<T> U;
        if (fwd) {
          LK::load(lk + size_t(par * 4 + mu) * LK::NC * Vh, Vh, blk * H + (ll >> 1), U);
          hop_fwd(mu, U, nb, kp * T(n.sign), f);
        } else {
          LK::load(lk + size_t((1 - par) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
          hop_bwd(mu, U, nb, kp * T(n.sign), f);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q)
          fc[q][t] = make_float4(f.v[(2 * q) / 3][(2 * q) % 3].re, f.v[(2 * q) / 3][(2 * q) % 3].im,
                                 f.v[(2 * q + 1) / 3][(2 * q + 1) % 3].re, f.v[(2 * q + 1) / 3][(2 * q + 1) % 3].im);
      };
      // waves 0-3 take directions 0, 0, 1, 1 (forward, backward in turn), then 2, 2, 3, 3
      const int t0 = int(threadIdx.x);
      if (__builtin_amdgcn_readfirstlane(t0 >> 7) == 0) {
        face_hop(std::integral_constant<int, 0>{}, t0);
        face_hop(std::integral_constant<int, 2>{}, t0 + 2 * H);
      } else {
        face_hop(std::integral_constant<int, 1>{}, t0);
        face_hop(std::integral_constant<int, 3>{}, t0 + 2 * H);
      }
      fetch_links();
      __syncthreads();
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        const int lm = lo[mu];
        if (lm == 3 || lm == 0) {
          int e = 0, c = 0;
#pragma unroll
          for (int m = 0; m < 4; ++m)
            if (m != mu) {
              e |= lo[m] << (2 * c);
              ++c;
            }
          const int t = mu * 128 + (lm == 3 ? 0 : 64) + e;
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const float4 v = fc[q][t];
            cx<T>& z0 = r.v[(2 * q) / 3][(2 * q) % 3];
            cx<T>& z1 = r.v[(2 * q + 1) / 3][(2 * q + 1) % 3];
            z0 = {z0.re + v.x, z0.im + v.y};
            z1 = {z1.re + v.z, z1.im + v.w};
          }
        }
      }
      __syncthreads();  // the links are staged over the face hops
    } else {
      if (a.face) face_update<S, LK, T>(g, lk, dl, h, s, kp, r);
      fetch_links();
    }
  } else if (a.face) {
    face_update<S, LK, T>(g, lk, dl, h, s, kp, r);
  }
  if constexpr (XH) {  // lane h stages kappa times the forward links of site j of parity h (whole, FP16)
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      SU3<float> U;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float4 v = lraw[mu * 3 + k];
        U.m[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
        U.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
      }
      su3_row2(U, 1.0f);
      uint32_t w[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) w[k] = h_pack(scale(kf, U.m[k / 3][k % 3]));
      const int i = (h * 4 + mu) * H + j;
      lk_a[i] = make_uint4(w[0], w[1], w[2], w[3]);
      lk_b[i] = make_uint4(w[4], w[5], w[6], w[7]);
      lk_c[i] = w[8];
    }
  }
  // forward link of site (parity gp, in-block index q) in direction mu
  auto link = [&](int mu, int gp, int q, int gs, SU3<T>& U) {
    if constexpr (LL) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        float4 v;
        if constexpr (LH) {
          const half4_t hv = __builtin_bit_cast(half4_t, lk_h[mu * 3 + k][gp * H + q]);
          v = make_float4(float(hv[0]), float(hv[1]), float(hv[2]), float(hv[3]));
        } else {
          v = lk_lds[mu * 3 + k][gp * H + q];
        }
        U.m[(2 * k) / 3][(2 * k) % 3] = {T(v.x), T(v.y)};
        U.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(v.z), T(v.w)};
      }
      su3_row2(U, T(ik));  // rows 0 and 1 carry kappa, their cross product kappa^2
    } else {
      LK::load(lk + size_t(gp * 4 + mu) * LK::NC * Vh, Vh, gs, U);
    }
  };
  // hop coefficient sg * kappa; with staged links kappa is in the link and the
  // coefficient is the constant sg = +-1, which folds into the additions
  auto coef = [&](auto sg) -> T {
    if constexpr (LL) return T(decltype(sg)::value);
    else return T(decltype(sg)::value) * kp;
  };
  using P1 = std::integral_constant<int, 1>;
  using M1 = std::integral_constant<int, -1>;
  // FP16 forms: link (gp, mu, q) and the spinor of site q of an exchange field
  auto link_h = [&](int mu, int gp, int q, SU3H& U) {
    const int i = (gp * 4 + mu) * H + q;
    const uint4 x = lk_a[i], y = lk_b[i];
    const uint32_t w[9] = {x.x, x.y, x.z, x.w, y.x, y.y, y.z, y.w, lk_c[i]};
#pragma unroll
    for (int k = 0; k < 9; ++k) U.m[k / 3][k % 3] = __builtin_bit_cast(h2_t, w[k]);
  };
  auto spinor_h = [&](const uint4 (*f)[H], int q, SpinorH& p) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const uint4 x = f[k][q];
      const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) p.v[(4 * k + e) / 3][(4 * k + e) % 3] = __builtin_bit_cast(h2_t, w[e]);
    }
  };
  // site j of the even (E = 0) or odd (E = 1) exchange field: put, add to, read
  auto put = [&](int E, const Spinor<T>& v) {
    if constexpr (XH) {
      uint4 (*f)[H] = E ? odh : evh;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        f[k][j] = make_uint4(h_pack(v.v[(4 * k) / 3][(4 * k) % 3]), h_pack(v.v[(4 * k + 1) / 3][(4 * k + 1) % 3]),
                             h_pack(v.v[(4 * k + 2) / 3][(4 * k + 2) % 3]), h_pack(v.v[(4 * k + 3) / 3][(4 * k + 3) % 3]));
    } else {
      cx<T>(*f)[NH] = E ? od : ev;
#pragma unroll
      for (int k = 0; k < 12; ++k) f[k][j] = v.v[k / 3][k % 3];
    }
  };
  auto get = [&](int E, Spinor<T>& v) {
    if constexpr (XH) {
      const uint4(*f)[H] = E ? odh : evh;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const uint4 x = f[k][j];
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) v.v[(4 * k + e) / 3][(4 * k + e) % 3] = h_unpack(w[e]);
      }
    } else {
      const cx<T>(*f)[NH] = E ? od : ev;
#pragma unroll
      for (int k = 0; k < 12; ++k) v.v[k / 3][k % 3] = f[k][j];
    }
  };
  // this lane's hops of site j of parity P (1: the odd site, applied to the even field;
  // 0: the even site, applied to the odd field)
  auto phase = [&](auto P, auto sg, Spinor<T>& acc) {
    constexpr int p = decltype(P)::value;
    const T c = coef(sg);
    zero(acc);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int q = p ? nA[mu] : nB[mu];
      if (q >= 0) {
        SU3<T> U;
        if (h == 0) link(mu, p, j, s, U);
        else link(mu, 1 - p, q, p ? gA[mu] : gB[mu], U);
        Spinor<T> nb;
#pragma unroll
        for (int k = 0; k < 12; ++k) nb.v[k / 3][k % 3] = p ? ev[k][q] : od[k][q];
        if (h == 0) hop_fwd(mu, U, nb, c, acc);
        else hop_bwd(mu, U, nb, c, acc);
      }
    }
  };
  // the same in the FP16 form, with sign SG and the hop sum in FP16 pairs
  auto phase_h = [&](auto P, auto sg, SpinorH& acc) {
    constexpr int p = decltype(P)::value;
    constexpr int SG = decltype(sg)::value;
#pragma unroll
    for (int k = 0; k < 12; ++k) acc.v[k / 3][k % 3] = h2_t{0, 0};
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int q = p ? nA[mu] : nB[mu];
      if (q >= 0) {
        SU3H U;
        if (h == 0) link_h(mu, p, j, U);  // U(x, mu) of site j
        else link_h(mu, 1 - p, q, U);     // U(x - mu, mu) of its neighbour
        SpinorH nb;
        spinor_h(p ? evh : odh, q, nb);
        if (h == 0) hoph_fwd<SG>(mu, U, nb, acc);
        else hoph_bwd<SG>(mu, U, nb, acc);
      }
    }
  };
  auto put_h = [&](int E, const SpinorH& v) {
    uint4(*f)[H] = E ? odh : evh;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) w[e] = __builtin_bit_cast(uint32_t, v.v[(4 * k + e) / 3][(4 * k + e) % 3]);
      f[k][j] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  };
  auto get_h = [&](int E, SpinorH& v) { spinor_h(E ? odh : evh, j, v); };
  auto phase_odd = [&](auto sg, Spinor<T>& acc) { phase(std::integral_constant<int, 1>{}, sg, acc); };
  auto phase_even = [&](auto sg, Spinor<T>& acc) { phase(std::integral_constant<int, 0>{}, sg, acc); };

  // |rho|^2 over the block
  double b2 = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) b2 += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
  b2 = wg_sum(b2, sm[0]);
  // FP16 exchange: work on sig * rho, with unit RMS per real component over the block
  const T sig = XH && b2 > 0.0 ? T(sqrt(double(24 * 2 * H) / b2)) : T(1);
  if constexpr (XH) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) r.v[q][c] = scale(sig, r.v[q][c]);
  }
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 * double(sig) * double(sig) : -1.0;
  zero(d);
  int it = 0;
  if constexpr (XH) {
    using P0 = std::integral_constant<int, 0>;
    using Q1 = std::integral_constant<int, 1>;
    SpinorH ah;
    // even right-hand side rho_e + k H_eo rho_o (lane 0); lane 1 keeps rho_o
    if (h == 1) put(1, r);
    __syncthreads();
    phase_h(P0{}, P1{}, ah);
    if (h == 1) put_h(0, ah);
    __syncthreads();
    if (h == 0) {
      SpinorH e;
      get_h(0, e);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<float> z = h_f32(ah.v[k / 3][k % 3] + e.v[k / 3][k % 3]);
        r.v[k / 3][k % 3] = {r.v[k / 3][k % 3].re + z.re, r.v[k / 3][k % 3].im + z.im};
      }
    }
    if (b2 > 0.0) {
      for (; it < a.niter; ++it) {
        // p = (1 - k^2 H_eo H_oe) r on the even sites
        if (h == 0) put(0, r);
        __syncthreads();
        phase_h(Q1{}, P1{}, ah);
        if (h == 0) put_h(1, ah);
        __syncthreads();
        if (h == 1) {
          SpinorH o;
          get_h(1, o);
#pragma unroll
          for (int k = 0; k < 12; ++k) o.v[k / 3][k % 3] = o.v[k / 3][k % 3] + ah.v[k / 3][k % 3];
          put_h(1, o);
        }
        __syncthreads();
        phase_h(P0{}, M1{}, ah);
        if (h == 1) put_h(0, ah);  // ev is free: every read of it was in the odd phase
        __syncthreads();
        // inner products summed in FP32 over the lane's twelve components, then in FP64
        float frr = 0.f, fri = 0.f, fpp = 0.f;
        if (h == 0) {
          SpinorH e;
          get_h(0, e);
#pragma unroll
          for (int k = 0; k < 12; ++k) {
            const cx<float> z = h_f32(ah.v[k / 3][k % 3] + e.v[k / 3][k % 3]);
            const cx<float> rv = r.v[k / 3][k % 3];
            const cx<float> pv = {rv.re + z.re, rv.im + z.im};
            acc.v[k / 3][k % 3] = pv;
            frr = fmadd(pv.re, rv.re, fmadd(pv.im, rv.im, frr));
            fri = fmadd(pv.re, rv.im, fmadd(-pv.im, rv.re, fri));
            fpp = fmadd(pv.re, pv.re, fmadd(pv.im, pv.im, fpp));
          }
        }
        double prr = frr, pri = fri, pp = fpp;
        wg_sum3(prr, pri, pp, sm);
        if (!(pp > 0.0)) break;
        const cx<T> alpha = {T(prr / pp), T(pri / pp)};
        float frs = 0.f;
        if (h == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
              r.v[q][c] = r.v[q][c] - cmul(alpha, acc.v[q][c]);
            }
          if (stop2 > 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
              for (int c = 0; c < 3; ++c) frs = fmadd(r.v[q][c].re, r.v[q][c].re, fmadd(r.v[q][c].im, r.v[q][c].im, frs));
          }
        }
        if (stop2 > 0) {
          const double rr = wg_sum(double(frs), sm[0]);
          if (rr <= stop2) {
            ++it;
            break;
          }
        }
      }
    }
    // x_o = rho_o + k H_oe x_e; the odd residual is then zero
    if (h == 0) put(0, d);
    __syncthreads();
    phase_h(Q1{}, P1{}, ah);
    if (h == 0) put_h(1, ah);
    __syncthreads();
    if (h == 1) {
      SpinorH o;
      get_h(1, o);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cx<float> z = h_f32(o.v[k / 3][k % 3] + ah.v[k / 3][k % 3]);
        d.v[k / 3][k % 3] = {r.v[k / 3][k % 3].re + z.re, r.v[k / 3][k % 3].im + z.im};
        r.v[k / 3][k % 3] = {T(0), T(0)};
      }
    }
  } else {

  // even right-hand side rho_e + k H_eo rho_o (lane 0); lane 1 keeps rho_o
  if (h == 1) put(1, r);
  __syncthreads();
  phase_even(P1{}, acc);
  if (h == 1) put(0, acc);
  __syncthreads();
  if (h == 0) {
    Spinor<T> e;
    get(0, e);
#pragma unroll
    for (int k = 0; k < 12; ++k) r.v[k / 3][k % 3] = r.v[k / 3][k % 3] + acc.v[k / 3][k % 3] + e.v[k / 3][k % 3];
  }

  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
      // p = (1 - k^2 H_eo H_oe) r on the even sites
      if (h == 0) put(0, r);
      __syncthreads();
      phase_odd(P1{}, acc);
      if (h == 0) put(1, acc);
      __syncthreads();
      if (h == 1) {
        Spinor<T> o;
        get(1, o);
#pragma unroll
        for (int k = 0; k < 12; ++k) o.v[k / 3][k % 3] = o.v[k / 3][k % 3] + acc.v[k / 3][k % 3];
        put(1, o);
      }
      __syncthreads();
      phase_even(M1{}, acc);
      if (h == 1) put(0, acc);  // ev is free: every read of it was in phase_odd
      __syncthreads();
      double prr = 0.0, pri = 0.0, pp = 0.0;
      if (h == 0) {
        Spinor<T> e;
        get(0, e);
#pragma unroll
        for (int k = 0; k < 12; ++k) acc.v[k / 3][k % 3] = r.v[k / 3][k % 3] + acc.v[k / 3][k % 3] + e.v[k / 3][k % 3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double ar = acc.v[q][c].re, ai = acc.v[q][c].im, br = r.v[q][c].re, bi = r.v[q][c].im;
            prr += ar * br + ai * bi;
            pri += ar * bi - ai * br;
            pp += ar * ar + ai * ai;
          }
      }
      wg_sum3(prr, pri, pp, sm);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
      if (h == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            d.v[q][c] = d.v[q][c] + cmul(alpha, r.v[q][c]);
            r.v[q][c] = r.v[q][c] - cmul(alpha, acc.v[q][c]);
            rr += double(r.v[q][c].re) * r.v[q][c].re + double(r.v[q][c].im) * r.v[q][c].im;
          }
      }
      if (stop2 > 0) {
        rr = wg_sum(rr, sm[0]);
        if (rr <= stop2) {
          ++it;
          break;
        }
      }
    }
  }
  // x_o = rho_o + k H_oe x_e; the odd residual is then zero
  if (h == 0) put(0, d);
  __syncthreads();
  phase_odd(P1{}, acc);
  if (h == 0) put(1, acc);
  __syncthreads();
  if (h == 1) {
    Spinor<T> o;
    get(1, o);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      d.v[k / 3][k % 3] = r.v[k / 3][k % 3] + o.v[k / 3][k % 3] + acc.v[k / 3][k % 3];
      r.v[k / 3][k % 3] = {T(0), T(0)};
    }
  }
  }
  if constexpr (XH) {  // back to the scale of rho
    const T isig = T(1) / sig;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        r.v[q][c] = scale(isig, r.v[q][c]);
        d.v[q][c] = scale(isig, d.v[q][c]);
      }
  }
  // the FP16 form's BF16 fields (the preconditioner's own residual, correction and
  // iterate) take the one-instruction conversion; other forms round to nearest even
  auto store = [&](unit* f, const Spinor<T>& v) {
    if constexpr (XH && std::is_same<S, StBF16>::value) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const cx<T> z = v.v[(4 * k + e) / 3][(4 * k + e) % 3];
          w[e] = bf16_pack2(z.re, z.im);
        }
        f[size_t(k) * Vh + s] = make_uint4(w[0], w[1], w[2], w[3]);
      }
    } else {
      S::store(f, Vh, s, v);
    }
  };
  store(rho + size_t(h) * S::NC * Vh, r);
  store(dl + size_t(h) * S::NC * Vh, d);
  Spinor<T> xv;
  if (a.x_assign) zero(xv);
  else S::load(x + size_t(h) * S::NC * Vh, Vh, s, xv);
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + d.v[q][c];
  store(x + size_t(h) * S::NC * Vh, xv);
  if (a.iters && threadIdx.x == 0) atomicMax(a.iters, it);
}

// Even-odd block solver for 256-site blocks with four lanes per site (512 threads,
// two waves per SIMD), for FP32 arithmetic. The algorithm is that of k_block_mr_eo;
// here each hop phase is spread four ways. Lane (j, m) takes the hops of site j in
// direction m & 1 (0 forward, 1 backward) along the dimension pair
// {2(m >> 1), 2(m >> 1) + 1} and writes its partial sum to LDS plane m; the four
// planes are summed afterwards. The solver state is spread as well: lane (j, m)
// holds the spinor components k = m, m + 4, m + 8 of the even and odd site j, so
// inner products and updates use every lane. With staged links the block's links
// are staged whole (row 2 rebuilt once) and pre-multiplied by kappa, so a hop
// neither rebuilds nor scales them.
template <class S, class LK, class T, bool STAGE>
__global__ void __launch_bounds__(512) k_block_mr_eo4(BlockArgs a) {
  constexpr int NL = 4;          // lanes per site
  constexpr int H = 128;         // sites per parity
  constexpr int NT = NL * H;     // threads
  constexpr int KC = 12 / NL;    // state components per lane
  static_assert(sizeof(T) == 4, "FP32 arithmetic (FP64 state does not fit the registers)");
  constexpr bool LL = LdsLinks<LK>::on && STAGE;  // whole kappa-scaled links in LDS
  __shared__ cx<T> fv[12][H];      // the field a hop phase reads
  __shared__ cx<T> pt[NL][12][H];  // partial sums of the lane groups
  __shared__ float4 lk_lds[LL ? 20 : 1][LL ? 2 * H : 1];  // 5 float4 per link
  __shared__ double sm[3][16];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const BlockCoord bc = block_coord(a);
  const int blk = bc.blk;
  const int prop = bc.prop;
  const size_t rix = size_t(prop * a.nrhs + bc.rhs);
  const size_t roff = rix * a.rhs_stride;
  using unit = typename S::unit;
  unit* rho = reinterpret_cast<unit*>(a.rho) + roff;
  unit* x = reinterpret_cast<unit*>(a.x) + roff;
  unit* dl = reinterpret_cast<unit*>(a.delta) + roff;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const T kp = T(a.kappa);
  const T ch = LL ? T(1) : kp;  // hop coefficient (kappa is in the staged links)
  const int t = threadIdx.x;
  const int j = t & (H - 1);
  const int m = __builtin_amdgcn_readfirstlane(t >> 7);
  const int h = m & 1;
  const int fp = m >> 1;  // parity of this lane's face update and stores
  const int s = blk * H + j;

  // global reads that depend on nothing else go first: this lane's rho (one lane per
  // site and parity), x (the lane that updates it), the links to stage
  Spinor<T> acc, xv;
  zero(acc);
  zero(xv);
  if (h == 0) load_rho0<S>(a, rho, rix, fp, s, acc);
  else if (!a.x_assign) S::load(x + size_t(fp) * S::NC * Vh, Vh, s, xv);
  // the site tables head the chain of dependent reads of the face update: read them
  // before the link staging so that their latency overlaps it
  SiteInfo so, se;
  site_info(g, 1, s, so);
  site_info(g, 0, s, se);
  if constexpr (LL) {  // link (parity gp, site q, mu) -> planes mu * 5 + e, kappa U
    for (int i = t; i < 4 * 2 * H; i += NT) {
      const int mu = i / (2 * H), xq = i - mu * 2 * H, gp = xq / H;
      SU3<T> U;
      LK::load(lk + size_t(gp * 4 + mu) * LK::NC * Vh, Vh, blk * H + (xq - gp * H), U);
      cx<T> e[10];
#pragma unroll
      for (int k = 0; k < 9; ++k) e[k] = scale(kp, U.m[k / 3][k % 3]);
      e[9] = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < 5; ++k)
        lk_lds[mu * 5 + k][xq] = make_float4(float(e[2 * k].re), float(e[2 * k].im), float(e[2 * k + 1].re), float(e[2 * k + 1].im));
    }
  }

  // in-block neighbours of this lane's hops: nA for the odd site j, nB for the even
  // site j (-1 when the hop leaves the block); gA, gB their indices in the field
  int nA[4], nB[4], gA[4], gB[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Nbr n = neighbour(g, so, mu, h == 0 ? +1 : -1);
    nA[mu] = n.cross ? -1 : n.s - blk * H;
    gA[mu] = n.s;
    Nbr q = neighbour(g, se, mu, h == 0 ? +1 : -1);
    nB[mu] = q.cross ? -1 : q.s - blk * H;
    gB[mu] = q.s;
  }
  auto link = [&](int mu, int gp, int q, int gs, SU3<T>& U) {
    if constexpr (LL) {
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        float4 v = lk_lds[mu * 5 + k][gp * H + q];
        U.m[(2 * k) / 3][(2 * k) % 3] = {T(v.x), T(v.y)};
        if (k < 4) U.m[(2 * k + 1) / 3][(2 * k + 1) % 3] = {T(v.z), T(v.w)};
      }
    } else {
      LK::load(lk + size_t(gp * 4 + mu) * LK::NC * Vh, Vh, gs, U);
    }
  };
  // kappa times this lane's hops of site j of parity gp (neighbours, of the other
  // parity, read from fv), into plane m
  auto phase = [&](int gp, const int (&nn)[4], const int (&gn)[4]) {
    Spinor<T> hs;
    zero(hs);
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if ((mu >> 1) != (m >> 1)) continue;  // wave-uniform
      const int q = nn[mu];
      if (q >= 0) {
        SU3<T> U;
        if (h == 0) link(mu, gp, j, s, U);    // U(x, mu)
        else link(mu, 1 - gp, q, gn[mu], U);  // U(x - mu, mu), stored at the neighbour
        const LdsSpinor<T, H> nb{{fv, q}};
        if (h == 0) hop_fwd(mu, U, nb, ch, hs);
        else hop_bwd(mu, U, nb, ch, hs);
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) pt[m][k][j] = hs.v[k / 3][k % 3];
  };
  // sum over all planes of component k of site j
  auto psum = [&](int k) {
    cx<T> v = pt[0][k][j];
#pragma unroll
    for (int q = 1; q < NL; ++q) v = v + pt[q][k][j];
    return v;
  };
  // spinor component held in this lane's state slot i
  auto comp = [&](int i) { return m + NL * i; };

  // rho of both parities with the face update, spread like the hops: plane m gets
  // the hops leaving the block from parity fp in direction h and, in one plane per
  // parity, rho itself. The reads are issued for every dimension at once, so their
  // latencies overlap: a hop that stays in the block reads a valid site (its own
  // index) and its spinor is replaced by zero, since that memory may hold anything,
  // NaN included, which a zero weight would not cancel.
  if (a.face) {
    const SiteInfo& si = fp ? so : se;
    const unit* dsrc = dl + size_t(1 - fp) * S::NC * Vh;
    SU3<T> U[4];
    Spinor<T> nb[4];
    T cf[4];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      Nbr n = neighbour(g, si, mu, h == 0 ? +1 : -1);
      const int ns = n.cross ? n.s : s;
      cf[mu] = n.cross ? kp * T(n.sign) : T(0);
      S::load(dsrc, Vh, ns, nb[mu]);
      if (h == 0) LK::load(lk + size_t(fp * 4 + mu) * LK::NC * Vh, Vh, s, U[mu]);
      else LK::load(lk + size_t((1 - fp) * 4 + mu) * LK::NC * Vh, Vh, ns, U[mu]);
#pragma unroll
      for (int k = 0; k < 12; ++k)
        if (!n.cross) nb[mu].v[k / 3][k % 3] = {T(0), T(0)};
    }
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if (h == 0) hop_fwd(mu, U[mu], nb[mu], cf[mu], acc);
      else hop_bwd(mu, U[mu], nb[mu], cf[mu], acc);
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) pt[m][k][j] = acc.v[k / 3][k % 3];
  __syncthreads();
  cx<T> r[KC], ro[KC], d[KC], ap[KC];
  double b2 = 0.0;
#pragma unroll
  for (int i = 0; i < KC; ++i) {
    const int k = comp(i);
    d[i] = ap[i] = {T(0), T(0)};
    r[i] = pt[0][k][j] + pt[1][k][j];  // planes 0, 1: parity 0; 2, 3: parity 1
    ro[i] = pt[2][k][j] + pt[3][k][j];
    b2 += double(r[i].re) * r[i].re + double(r[i].im) * r[i].im + double(ro[i].re) * ro[i].re +
          double(ro[i].im) * ro[i].im;
    fv[k][j] = ro[i];
  }
  b2 = wg_sum(b2, sm[0]);  // its barriers also publish fv and free pt
  const double stop2 = a.tol > 0 ? a.tol * a.tol * b2 : -1.0;

  // even right-hand side rho_e + k H_eo rho_o
  phase(0, nB, gB);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KC; ++i)
    r[i] = r[i] + psum(comp(i));

  int it = 0;
  if (b2 > 0.0) {
    for (; it < a.niter; ++it) {
      // ap = (1 - k^2 H_eo H_oe) r on the even sites
#pragma unroll
      for (int i = 0; i < KC; ++i)
        fv[comp(i)][j] = r[i];
      __syncthreads();
      phase(1, nA, gA);
      __syncthreads();
#pragma unroll
      for (int i = 0; i < KC; ++i)
        fv[comp(i)][j] = psum(comp(i));
      __syncthreads();
      phase(0, nB, gB);
      __syncthreads();
      double prr = 0.0, pri = 0.0, pp = 0.0;
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        {
          ap[i] = r[i] - psum(comp(i));
          const double ar = ap[i].re, ai = ap[i].im, br = r[i].re, bi = r[i].im;
          prr += ar * br + ai * bi;
          pri += ar * bi - ai * br;
          pp += ar * ar + ai * ai;
        }
      }
      wg_sum3(prr, pri, pp, sm);
      if (!(pp > 0.0)) break;
      const cx<T> alpha = {T(prr / pp), T(pri / pp)};
      double rr = 0.0;
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        d[i] = d[i] + cmul(alpha, r[i]);
        r[i] = r[i] - cmul(alpha, ap[i]);
        rr += double(r[i].re) * r[i].re + double(r[i].im) * r[i].im;
      }
      if (stop2 > 0) {
        rr = wg_sum(rr, sm[0]);
        if (rr <= stop2) {
          ++it;
          break;
        }
      }
    }
  }
  // x_o = rho_o + k H_oe x_e; the odd residual is then zero
#pragma unroll
  for (int i = 0; i < KC; ++i)
    fv[comp(i)][j] = d[i];
  __syncthreads();
  phase(1, nA, gA);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < KC; ++i)
    ro[i] = ro[i] + psum(comp(i));
  __syncthreads();
  // gather the even residual (plane 0), even delta (plane 1) and odd delta (plane 2)
  // per site, then store whole spinors: lane group m = 0 rho_e, 1 delta_e and x_e,
  // 2 rho_o (zero), 3 delta_o and x_o
#pragma unroll
  for (int i = 0; i < KC; ++i) {
    pt[0][comp(i)][j] = r[i];
    pt[1][comp(i)][j] = d[i];
    pt[2][comp(i)][j] = ro[i];
  }
  __syncthreads();
  {
    Spinor<T> v;
    if (m == 2) zero(v);
    else {
      const int plane = m == 0 ? 0 : (m == 1 ? 1 : 2);
#pragma unroll
      for (int k = 0; k < 12; ++k) v.v[k / 3][k % 3] = pt[plane][k][j];
    }
    if (h == 0) {
      S::store(rho + size_t(fp) * S::NC * Vh, Vh, s, v);
    } else {
      S::store(dl + size_t(fp) * S::NC * Vh, Vh, s, v);
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) xv.v[q][c] = xv.v[q][c] + v.v[q][c];
      S::store(x + size_t(fp) * S::NC * Vh, Vh, s, xv);
    }
  }
  if (a.iters && t == 0) atomicMax(a.iters, it);
}

template <class S, class LK, class T>
static void block_go(hipStream_t st, const BlockArgs& a, int nprop) {
  if (2 * a.g.Vbh == 256) {
    const dim3 grid(a.g.nblk_c, a.nrhs, nprop);
    if (a.eo) {
      // links staged in LDS (eo 1) or read from L2 (eo 2); in FP32 2 or 4 lanes per
      // site, by default 4 when the grid leaves compute units idle (the iteration's
      // latency then sets the time, and four lanes halve the hops per lane), else 2
      // (fewer barriers and LDS passes when the CUs are full). FP64 uses 2.
      constexpr bool LL = LdsLinks<LK>::on;
      const bool stage = a.eo != 2;
      if constexpr (sizeof(T) == 4) {
        const int nl = a.eo_lanes > 0 ? a.eo_lanes : (grid.x * grid.y * grid.z < 256 ? 4 : 2);
        if (nl == 4) {
          if (LL && stage) launch_timed((k_block_mr_eo4<S, LK, T, true>), grid, dim3(512), 0, st, a);
          else launch_timed((k_block_mr_eo4<S, LK, T, false>), grid, dim3(512), 0, st, a);
          return;
        }
      }
      if (LL && !stage) launch_timed((k_block_mr_eo<S, LK, T, false>), grid, dim3(256), 0, st, a);
      else if (LL && a.link16 == 2 && sizeof(T) == 4) launch_timed((k_block_mr_eo<S, LK, T, true, 2>), grid, dim3(256), 0, st, a);
      else if (LL && a.link16) launch_timed((k_block_mr_eo<S, LK, T, true, 1>), grid, dim3(256), 0, st, a);
      else launch_timed((k_block_mr_eo<S, LK, T>), grid, dim3(256), 0, st, a);
      return;
    }
    if constexpr (LdsLinks<LK>::on) {
      // two lanes per site when the grid gives fewer than two workgroups per CU
      const int lanes = a.lanes > 0 ? a.lanes : (grid.x * grid.y * grid.z < 512 ? 2 : 1);
      if (lanes == 2) {
        launch_timed((k_block_mr_lds2<S, LK, T>), grid, dim3(512), 0, st, a);
        return;
      }
    }
    launch_timed((k_block_mr_lds<S, LK, T, 256>), grid, dim3(256), 0, st, a);
    return;
  }
  dim3 grid(a.g.nblk_c, a.nrhs, nprop);
  if (a.eo) {
    const int threads = a.g.Vbh < 256 ? ((a.g.Vbh + 63) / 64) * 64 : 256;
    launch_timed((k_block_mr_eo_g<S, LK, T>), grid, dim3(threads), 0, st, a);
    return;
  }
  int threads = 2 * a.g.Vbh < 256 ? ((2 * a.g.Vbh + 63) / 64) * 64 : 256;
  launch_timed((k_block_mr<S, LK, T>), grid, dim3(threads), 0, st, a);
}

void launch_block_mr(hipStream_t st, const Geo& g, const void* const* links, int linkfmt, const FieldBatch& rho,
                     const FieldBatch& x, const FieldBatch& delta, const FieldBatch& pbuf, const BlockMRParams& bp,
                     int* iters_out) {
  BlockArgs a;
  a.g = g;
  for (int i = 0; i < MAXPROP; ++i) a.links[i] = i < rho.nprop ? links[i] : nullptr;
  a.rho = rho.p;
  a.x = x.p;
  a.delta = delta.p;
  a.pbuf = pbuf.p;
  a.rhs_stride = units_per_field(rho.prec, g.Vh);
  a.nrhs = rho.nrhs;
  a.colour = bp.colour;
  a.niter = bp.niter;
  a.tol = bp.tol;
  a.kappa = bp.kappa;
  a.face = bp.face;
  a.lanes = bp.lanes;
  a.eo = bp.eo;
  a.rho_in = bp.rho_in;
  a.x_assign = bp.x_assign;
  a.eo_lanes = bp.eo_lanes;
  a.xcd_map = bp.xcd_map;
  a.rin_f32 = bp.rho_in_f32;
  a.link16 = bp.link16;
  a.rin_stride = units_per_field(P_F32, g.Vh);
  a.iters = iters_out;
  if (rho.prec == P_F64 && linkfmt == LK_F64) block_go<StF64, LkF64, double>(st, a, rho.nprop);
  else if (rho.prec == P_F32 && linkfmt == LK_F32C12) block_go<StF32, LkF32C12, float>(st, a, rho.nprop);
  else if (rho.prec == P_BF16 && linkfmt == LK_F32C12) block_go<StBF16, LkF32C12, float>(st, a, rho.nprop);
  else if (rho.prec == P_F32 && linkfmt == LK_F32F18) block_go<StF32, LkF32F18, float>(st, a, rho.nprop);
  else if (rho.prec == P_BF16 && linkfmt == LK_F32F18) block_go<StBF16, LkF32F18, float>(st, a, rho.nprop);
}

}  // namespace psms
