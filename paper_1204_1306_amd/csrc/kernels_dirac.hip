// Wilson-Dirac stencil kernels (eq. Dw), the Schur projector P (Sec. 4.4) and
// the boundary <-> internal layout conversions.
#include "kernels.h"

namespace psms {

size_t units_per_field(Prec prec, int Vh) {
  int nc = prec == P_F64 ? 12 : prec == P_F32 ? 6 : 3;
  return size_t(2) * nc * Vh;
}
size_t bytes_per_field(Prec prec, int Vh) { return units_per_field(prec, Vh) * 16; }

// ----------------------------------------------------------------- stencil
struct DslashArgs {
  Geo g;
  const void* links[MAXPROP];
  const void* in;
  void* out;
  size_t in_rhs_stride, out_rhs_stride;  // units
  int nrhs;                              // per proposal
  int p0, np, blk0, nb;
  double cdiag, chop;
  int accumulate;
  int xcd_map;  // 1: remap workgroups to per-XCD contiguous tile ranges
  int nt_out;   // 1: non-temporal output stores (output larger than the chip's L2)
};

// Workgroup -> site tile. Workgroups are dispatched round-robin over the 8 XCDs,
// so workgroup w is given tile q = (w % 8) * (nwg / 8) + w / 8: every XCD sweeps a
// contiguous slab of tiles and keeps its neighbours in its own L2. Inside the
// sweep the two parities alternate tile by tile and, when all blocks are
// processed, the blocks follow the host-built schedule g.border (black block bi,
// then white block bi: neighbours along direction 3), so that the data one tile
// reads is the data the next one needs.
__device__ __forceinline__ bool tile_site(const DslashArgs& a, int& p, int& s) {
  const Geo& g = a.g;
  const int nwg = gridDim.x;
  const int w = blockIdx.x;
  const int q = (a.xcd_map && (nwg & 7) == 0) ? (w & 7) * (nwg >> 3) + (w >> 3) : w;
  const int tpp = (a.nb * g.Vbh + 255) >> 8;  // tiles per parity
  const int tp = q % a.np;
  const int tq = q / a.np;
  if (tq >= tpp) return false;
  const int o = (tq << 8) + threadIdx.x;
  if (o >= a.nb * g.Vbh) return false;
  p = a.p0 + tp;
  if (a.nb == g.nblk) {
    const int bp = o / g.Vbh;
    s = g.border[bp] * g.Vbh + (o - bp * g.Vbh);
  } else {
    s = a.blk0 * g.Vbh + o;
  }
  return true;
}

template <class SI, class SO, class LK, class T, int SEL, int NR, int W = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_dslash(DslashArgs a) {
  const Geo& g = a.g;
  int p, s;
  if (!tile_site(a, p, s)) return;
  const int prop = blockIdx.z;
  const int rhs0 = blockIdx.y * NR;
  const int nr = min(NR, a.nrhs - rhs0);
  const size_t Vh = g.Vh;

  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const typename SI::unit* in = reinterpret_cast<const typename SI::unit*>(a.in) + size_t(prop * a.nrhs + rhs0) * a.in_rhs_stride;
  typename SO::unit* out = reinterpret_cast<typename SO::unit*>(a.out) + size_t(prop * a.nrhs + rhs0) * a.out_rhs_stride;

  SiteInfo si;
  site_info(g, p, s, si);

  // the diagonal term seeds the accumulator: the site's own spinor is read first,
  // close in time to the neighbouring tile's reads of the same lines
  Spinor<T> acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (a.cdiag != 0.0 && r < nr) {
      SI::load(in + r * a.in_rhs_stride + size_t(p) * SI::NC * Vh, Vh, s, acc[r]);
      const T cd = T(a.cdiag);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[r].v[sp][c] = scale(cd, acc[r].v[sp][c]);
    } else {
      zero(acc[r]);
    }
  }

  const T ch = T(a.chop);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    // forward hop: U(x,mu) (1 - gamma_mu) psi(x + mu)
    {
      Nbr n = neighbour(g, si, mu, +1);
      bool use = SEL == HOP_ALL || (SEL == HOP_INTRA ? !n.cross : n.cross);
      if (use) {
        SU3<T> U;
        LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            Spinor<T> nb;
            SI::load(in + r * a.in_rhs_stride + size_t(1 - p) * SI::NC * Vh, Vh, n.s, nb);
            hop_fwd(mu, U, nb, ch * T(n.sign), acc[r]);
          }
        }
      }
    }
    // backward hop: U(x - mu, mu)^+ (1 + gamma_mu) psi(x - mu)
    {
      Nbr n = neighbour(g, si, mu, -1);
      bool use = SEL == HOP_ALL || (SEL == HOP_INTRA ? !n.cross : n.cross);
      if (use) {
        SU3<T> U;
        LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          if (r < nr) {
            Spinor<T> nb;
            SI::load(in + r * a.in_rhs_stride + size_t(1 - p) * SI::NC * Vh, Vh, n.s, nb);
            hop_bwd(mu, U, nb, ch * T(n.sign), acc[r]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    if (r < nr) {
      typename SO::unit* o = out + r * a.out_rhs_stride + size_t(p) * SO::NC * Vh;
      if (a.accumulate) {
        Spinor<T> d;
        SO::load(o, Vh, s, d);
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[r].v[sp][c] = acc[r].v[sp][c] + d.v[sp][c];
      }
      if (a.nt_out) SO::store_nt(o, Vh, s, acc[r]);
      else SO::store(o, Vh, s, acc[r]);
    }
  }
}

// Split form of the full-lattice stencil (see k_dslash_split).
template <class SI, class SO, class LK, class T, int W = 1>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_dslash_split(DslashArgs a) {
  // 128 sites per workgroup; waves 0-1 sum the forward hops, waves 2-3 the backward
  // hops of the same sites (wave-uniform branch), the halves meet in LDS.
  __shared__ cx<T> part[12][128];
  const Geo& g = a.g;
  const int nwg = gridDim.x;
  const int w = blockIdx.x;
  const int q = (a.xcd_map && (nwg & 7) == 0) ? (w & 7) * (nwg >> 3) + (w >> 3) : w;
  const int tpp = (a.nb * g.Vbh + 127) >> 7;
  const int tp = q % a.np;
  const int tq = q / a.np;
  const int h = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7);  // wave-uniform
  const int l = threadIdx.x & 127;
  const int o = (tq << 7) + l;
  const bool valid = tq < tpp && o < a.nb * g.Vbh;
  int p = a.p0 + tp, s = 0;
  if (valid) {
    if (a.nb == g.nblk) {
      const int bp = o / g.Vbh;
      s = g.border[bp] * g.Vbh + (o - bp * g.Vbh);
    } else {
      s = a.blk0 * g.Vbh + o;
    }
  }
  const int prop = blockIdx.z;
  const size_t Vh = g.Vh;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const typename SI::unit* in = reinterpret_cast<const typename SI::unit*>(a.in) + size_t(prop * a.nrhs + blockIdx.y) * a.in_rhs_stride;
  typename SO::unit* out = reinterpret_cast<typename SO::unit*>(a.out) + size_t(prop * a.nrhs + blockIdx.y) * a.out_rhs_stride;
  Spinor<T> acc;
  zero(acc);
  if (valid) {
    SiteInfo si;
    site_info(g, p, s, si);
    const T ch = T(a.chop);
    const typename SI::unit* nin = in + size_t(1 - p) * SI::NC * Vh;
    if (h == 0 && a.cdiag != 0.0) {
      SI::load(in + size_t(p) * SI::NC * Vh, Vh, s, acc);
      const T cd = T(a.cdiag);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.v[sp][c] = scale(cd, acc.v[sp][c]);
    }
    if (h == 0) {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        Nbr n = neighbour(g, si, mu, +1);
        SU3<T> U;
        LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
        Spinor<T> nb;
        SI::load(nin, Vh, n.s, nb);
        hop_fwd(mu, U, nb, ch * T(n.sign), acc);
      }
    } else {
#pragma unroll
      for (int mu = 0; mu < 4; ++mu) {
        Nbr n = neighbour(g, si, mu, -1);
        SU3<T> U;
        LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
        Spinor<T> nb;
        SI::load(nin, Vh, n.s, nb);
        hop_bwd(mu, U, nb, ch * T(n.sign), acc);
      }
    }
  }
  if (h == 1) {
#pragma unroll
    for (int k = 0; k < 12; ++k) part[k][l] = acc.v[k / 3][k % 3];
  }
  __syncthreads();
  if (h == 1 || !valid) return;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc.v[k / 3][k % 3] = acc.v[k / 3][k % 3] + part[k][l];
  typename SO::unit* op = out + size_t(p) * SO::NC * Vh;
  if (a.accumulate) {
    Spinor<T> d;
    SO::load(op, Vh, s, d);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sp][c] = acc.v[sp][c] + d.v[sp][c];
  }
  if (a.nt_out) SO::store_nt(op, Vh, s, acc);
  else SO::store(op, Vh, s, acc);
}

template <class SI, class SO, class LK, class T, int W>
static void dslash_split_go(hipStream_t st, const DslashArgs& a, int nprop) {
  int tiles = a.np * ((a.nb * a.g.Vbh + 127) / 128);
  dim3 grid(tiles, a.nrhs, nprop);
  launch_timed((k_dslash_split<SI, SO, LK, T, W>), grid, dim3(256), 0, st, a);
}

template <class SI, class SO, class LK, class T, int W>
static void dslash_one_go(hipStream_t st, const DslashArgs& a, int nprop) {
  int tiles = a.np * ((a.nb * a.g.Vbh + 255) / 256);
  dim3 grid(tiles, a.nrhs, nprop);
  launch_timed((k_dslash<SI, SO, LK, T, HOP_ALL, 1, W>), grid, dim3(256), 0, st, a);
}

// Four lanes per site: 64 sites per workgroup; wave q takes two of the eight hops
// (q = 0: forward mu 0,1; 1: forward mu 2,3; 2: backward mu 0,1; 3: backward mu 2,3),
// wave 0 also the diagonal term; the partial sums meet in LDS. A lane holds the loads
// of only two hops, so two waves fit on a SIMD and interleave their memory latency.
template <class SI, class SO, class LK, class T, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_dslash_quad(DslashArgs a) {
  __shared__ cx<T> part[3][12][64];
  const Geo& g = a.g;
  const int nwg = gridDim.x;
  const int w = blockIdx.x;
  const int qq = (a.xcd_map && (nwg & 7) == 0) ? (w & 7) * (nwg >> 3) + (w >> 3) : w;
  const int tpp = (a.nb * g.Vbh + 63) >> 6;
  const int tp = qq % a.np;
  const int tq = qq / a.np;
  const int q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int l = threadIdx.x & 63;
  const int o = (tq << 6) + l;
  const bool valid = tq < tpp && o < a.nb * g.Vbh;
  const int p = a.p0 + tp;
  int s = 0;
  if (valid) {
    if (a.nb == g.nblk) {
      const int bp = o / g.Vbh;
      s = g.border[bp] * g.Vbh + (o - bp * g.Vbh);
    } else {
      s = a.blk0 * g.Vbh + o;
    }
  }
  const int prop = blockIdx.z;
  const size_t Vh = g.Vh;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const typename SI::unit* in = reinterpret_cast<const typename SI::unit*>(a.in) + size_t(prop * a.nrhs + blockIdx.y) * a.in_rhs_stride;
  typename SO::unit* out = reinterpret_cast<typename SO::unit*>(a.out) + size_t(prop * a.nrhs + blockIdx.y) * a.out_rhs_stride;
  Spinor<T> acc;
  zero(acc);
  if (valid) {
    SiteInfo si;
    site_info(g, p, s, si);
    const T ch = T(a.chop);
    const typename SI::unit* nin = in + size_t(1 - p) * SI::NC * Vh;
    if (q == 0 && a.cdiag != 0.0) {
      SI::load(in + size_t(p) * SI::NC * Vh, Vh, s, acc);
      const T cd = T(a.cdiag);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.v[sp][c] = scale(cd, acc.v[sp][c]);
    }
    // directions as compile-time constants, chosen by a wave-uniform test
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      if ((mu >> 1) != (q & 1)) continue;
      if (q < 2) {
        Nbr n = neighbour(g, si, mu, +1);
        SU3<T> U;
        LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
        Spinor<T> nb;
        SI::load(nin, Vh, n.s, nb);
        hop_fwd(mu, U, nb, ch * T(n.sign), acc);
      } else {
        Nbr n = neighbour(g, si, mu, -1);
        SU3<T> U;
        LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
        Spinor<T> nb;
        SI::load(nin, Vh, n.s, nb);
        hop_bwd(mu, U, nb, ch * T(n.sign), acc);
      }
    }
  }
  if (q > 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) part[q - 1][k][l] = acc.v[k / 3][k % 3];
  }
  __syncthreads();
  if (q > 0 || !valid) return;
#pragma unroll
  for (int k = 0; k < 12; ++k)
    acc.v[k / 3][k % 3] = acc.v[k / 3][k % 3] + part[0][k][l] + part[1][k][l] + part[2][k][l];
  typename SO::unit* op = out + size_t(p) * SO::NC * Vh;
  if (a.accumulate) {
    Spinor<T> d;
    SO::load(op, Vh, s, d);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sp][c] = acc.v[sp][c] + d.v[sp][c];
  }
  if (a.nt_out) SO::store_nt(op, Vh, s, acc);
  else SO::store(op, Vh, s, acc);
}

template <class SI, class SO, class LK, class T, int W>
static void dslash_quad_go(hipStream_t st, const DslashArgs& a, int nprop) {
  int tiles = a.np * ((a.nb * a.g.Vbh + 63) / 64);
  dim3 grid(tiles, a.nrhs, nprop);
  launch_timed((k_dslash_quad<SI, SO, LK, T, W>), grid, dim3(256), 0, st, a);
}

// Workgroup -> (position in the block schedule, right-hand side, proposal) for the
// one-workgroup-per-block forms (7, 8), whose grid is (blocks, right-hand sides,
// proposals). Workgroups go to the 8 XCDs in turn by linear index w; with xcd_map, w
// is read as XCD w % 8 and position w / 8 on it: each XCD takes a contiguous range of
// the schedule and runs the right-hand sides of one block back to back, so that they
// find that block's links in its L2.
struct TileCoord {
  int q, rhs, prop;
};
__device__ __forceinline__ TileCoord tile_coord(const DslashArgs& a) {
  const int nb = gridDim.x, nr = gridDim.y, np = gridDim.z;
  if (a.xcd_map && ((nb * np) & 7) == 0) {
    const int w = blockIdx.x + nb * (blockIdx.y + nr * blockIdx.z);
    const int i = w >> 3;
    const int q = (w & 7) * ((nb * np) >> 3) + i / nr;
    return {q % nb, i % nr, q / nb};
  }
  return {int(blockIdx.x), int(blockIdx.y), int(blockIdx.z)};
}

// Block-tile form (variant 7) for blocks of at most 256 sites: one workgroup per block,
// one lane per site of either parity. The block's input spinor (both parities) is read
// once into LDS; a hop that stays in the block reads its neighbour from there and only
// the hops that leave the block read the neighbour's spinor from memory. This cuts the
// L1 -> L2 requests per site, which bound the one-lane forms.
template <class SI, class SO, class LK, class T, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_dslash_block(DslashArgs a) {
  __shared__ cx<T> sp[2][12][128];
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const int Vbh = g.Vbh;
  const TileCoord tc = tile_coord(a);
  const int blk = g.border[tc.q];
  const int t = threadIdx.x;
  const int p = t >= Vbh ? 1 : 0;
  const int i = t - p * Vbh;
  const bool active = t < 2 * Vbh;
  const int s = blk * Vbh + i;
  const int prop = tc.prop;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const typename SI::unit* in = reinterpret_cast<const typename SI::unit*>(a.in) + size_t(prop * a.nrhs + tc.rhs) * a.in_rhs_stride;
  typename SO::unit* out = reinterpret_cast<typename SO::unit*>(a.out) + size_t(prop * a.nrhs + tc.rhs) * a.out_rhs_stride;

  Spinor<T> acc;
  if (active) {
    SI::load(in + size_t(p) * SI::NC * Vh, Vh, s, acc);
#pragma unroll
    for (int k = 0; k < 12; ++k) sp[p][k][i] = acc.v[k / 3][k % 3];
  }
  __syncthreads();
  if (!active) return;  // no barrier follows
  const T cd = T(a.cdiag), ch = T(a.chop);
#pragma unroll
  for (int sc = 0; sc < 4; ++sc)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.v[sc][c] = scale(cd, acc.v[sc][c]);
  SiteInfo si;
  site_info(g, p, s, si);
  const cx<T>(*nbr)[128] = sp[1 - p];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    {  // forward hop: U(x,mu) (1 - gamma_mu) psi(x + mu)
      Nbr n = neighbour(g, si, mu, +1);
      SU3<T> U;
      LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
      if (!n.cross) {
        const LdsSpinor<T, 128> nb{{nbr, n.s - blk * Vbh}};
        hop_fwd(mu, U, nb, ch, acc);
      } else {
        Spinor<T> nb;
        SI::load(in + size_t(1 - p) * SI::NC * Vh, Vh, n.s, nb);
        hop_fwd(mu, U, nb, ch * T(n.sign), acc);
      }
    }
    {  // backward hop: U(x - mu, mu)^+ (1 + gamma_mu) psi(x - mu)
      Nbr n = neighbour(g, si, mu, -1);
      SU3<T> U;
      LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, n.s, U);
      if (!n.cross) {
        const LdsSpinor<T, 128> nb{{nbr, n.s - blk * Vbh}};
        hop_bwd(mu, U, nb, ch, acc);
      } else {
        Spinor<T> nb;
        SI::load(in + size_t(1 - p) * SI::NC * Vh, Vh, n.s, nb);
        hop_bwd(mu, U, nb, ch * T(n.sign), acc);
      }
    }
  }
  typename SO::unit* op = out + size_t(p) * SO::NC * Vh;
  if (a.accumulate) {
    Spinor<T> d;
    SO::load(op, Vh, s, d);
#pragma unroll
    for (int sc = 0; sc < 4; ++sc)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sc][c] = acc.v[sc][c] + d.v[sc][c];
  }
  if (a.nt_out) SO::store_nt(op, Vh, s, acc);
  else SO::store(op, Vh, s, acc);
}

template <class SI, class SO, class LK, class T, int W>
static void dslash_block_go(hipStream_t st, const DslashArgs& a, int nprop) {
  dim3 grid(a.g.nblk, a.nrhs, nprop);
  launch_timed((k_dslash_block<SI, SO, LK, T, W>), grid, dim3(256), 0, st, a);
}

// Block-tile form with exchange (variant 8) for blocks of at most 256 sites: one
// workgroup per block, one lane per site of either parity, as variant 7, but every
// link and every in-block spinor is read from memory once per block. Direction by
// direction, the lane of site y loads its own forward link U(y,mu) and uses it twice:
// for its own forward hop, with psi(y + mu) read from the block's spinors in LDS, and
// for the backward hop of its neighbour y + mu, U(y,mu)^+ (1 + gamma_mu) psi(y), whose
// two colour vectors it leaves in LDS for that neighbour. Only the hops that leave the
// block read from memory: the neighbour's spinor, and for a backward hop its link.
template <class SI, class SO, class LK, class T, int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_dslash_tile(DslashArgs a) {
  __shared__ cx<T> sp[2][12][128];  // the block's input spinor, both parities
  __shared__ cx<T> hb[2][6][128];   // backward half spinors, by the receiving site
  const Geo& g = a.g;
  const size_t Vh = g.Vh;
  const int Vbh = g.Vbh;
  const TileCoord tc = tile_coord(a);
  const int blk = g.border[tc.q];
  const int t = threadIdx.x;
  const int p = t >= Vbh ? 1 : 0;
  const int i = t - p * Vbh;
  const bool active = t < 2 * Vbh;
  const int s = blk * Vbh + i;
  const int prop = tc.prop;
  const typename LK::unit* lk = reinterpret_cast<const typename LK::unit*>(a.links[prop]);
  const typename SI::unit* in = reinterpret_cast<const typename SI::unit*>(a.in) + size_t(prop * a.nrhs + tc.rhs) * a.in_rhs_stride;
  typename SO::unit* out = reinterpret_cast<typename SO::unit*>(a.out) + size_t(prop * a.nrhs + tc.rhs) * a.out_rhs_stride;
  const typename SI::unit* nin = in + size_t(1 - p) * SI::NC * Vh;

  Spinor<T> acc;
  zero(acc);
  SiteInfo si;
  if (active) {
    SI::load(in + size_t(p) * SI::NC * Vh, Vh, s, acc);
#pragma unroll
    for (int k = 0; k < 12; ++k) sp[p][k][i] = acc.v[k / 3][k % 3];
    const T cd = T(a.cdiag);
#pragma unroll
    for (int sc = 0; sc < 4; ++sc)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sc][c] = scale(cd, acc.v[sc][c]);
    site_info(g, p, s, si);
  }
  const T ch = T(a.chop);
  const LdsSpinor<T, 128> own{{sp[p], i}};
  __syncthreads();
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    Nbr nf, nb;
    if (active) {
      nf = neighbour(g, si, mu, +1);
      nb = neighbour(g, si, mu, -1);
      SU3<T> U;
      LK::load(lk + size_t(p * 4 + mu) * LK::NC * Vh, Vh, s, U);
      if (!nf.cross) {
        const int r = nf.s - blk * Vbh;
        cx<T> w0[3], w1[3];
        bwd_half(mu, U, own, w0, w1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          hb[1 - p][c][r] = w0[c];
          hb[1 - p][3 + c][r] = w1[c];
        }
        const LdsSpinor<T, 128> v{{sp[1 - p], r}};
        hop_fwd(mu, U, v, ch, acc);
      } else {
        Spinor<T> v;
        SI::load(nin, Vh, nf.s, v);
        hop_fwd(mu, U, v, ch * T(nf.sign), acc);
      }
    }
    __syncthreads();
    if (active) {
      if (!nb.cross) {
        cx<T> w0[3], w1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          w0[c] = hb[p][c][i];
          w1[c] = hb[p][3 + c][i];
        }
        bwd_recon(mu, w0, w1, ch, acc);
      } else {
        SU3<T> U;
        LK::load(lk + size_t((1 - p) * 4 + mu) * LK::NC * Vh, Vh, nb.s, U);
        Spinor<T> v;
        SI::load(nin, Vh, nb.s, v);
        hop_bwd(mu, U, v, ch * T(nb.sign), acc);
      }
    }
    if (mu < 3) __syncthreads();  // hb is written again by the next direction
  }
  if (!active) return;
  typename SO::unit* op = out + size_t(p) * SO::NC * Vh;
  if (a.accumulate) {
    Spinor<T> d;
    SO::load(op, Vh, s, d);
#pragma unroll
    for (int sc = 0; sc < 4; ++sc)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.v[sc][c] = acc.v[sc][c] + d.v[sc][c];
  }
  if (a.nt_out) SO::store_nt(op, Vh, s, acc);
  else SO::store(op, Vh, s, acc);
}

template <class SI, class SO, class LK, class T, int W>
static void dslash_tile_go(hipStream_t st, const DslashArgs& a, int nprop) {
  dim3 grid(a.g.nblk, a.nrhs, nprop);
  launch_timed((k_dslash_tile<SI, SO, LK, T, W>), grid, dim3(256), 0, st, a);
}

// Full-lattice stencil variants (form x register budget), chosen by the autotuner:
//   0: one lane per site          1: two wave groups per site
//   2: one lane, >= 4 waves/SIMD  3: split, >= 4 waves/SIMD
//   4: one lane, >= 6 waves/SIMD  5: split, >= 6 waves/SIMD
//   6: four lanes per site, >= 2 waves/SIMD
//   7: one workgroup per block of <= 256 sites, the block's input spinor in LDS
//   8: as 7, each link read once per block and the backward hops handed on in LDS
//      (7, 8: other block sizes, or part of the lattice: variant 0)
template <class SI, class SO, class LK, class T>
static void dslash_variant(hipStream_t st, const DslashArgs& a, int nprop, int v) {
  if (v >= 7 && !(2 * a.g.Vbh <= 256 && a.np == 2 && a.p0 == 0 && a.nb == a.g.nblk)) v = 0;
  switch (v) {
    case 8: dslash_tile_go<SI, SO, LK, T, 1>(st, a, nprop); break;
    case 7: dslash_block_go<SI, SO, LK, T, 1>(st, a, nprop); break;
    case 1: dslash_split_go<SI, SO, LK, T, 1>(st, a, nprop); break;
    case 2: dslash_one_go<SI, SO, LK, T, 4>(st, a, nprop); break;
    case 3: dslash_split_go<SI, SO, LK, T, 4>(st, a, nprop); break;
    case 4: dslash_one_go<SI, SO, LK, T, 6>(st, a, nprop); break;
    case 5: dslash_split_go<SI, SO, LK, T, 6>(st, a, nprop); break;
    case 6: dslash_quad_go<SI, SO, LK, T, 2>(st, a, nprop); break;
    default: dslash_one_go<SI, SO, LK, T, 1>(st, a, nprop); break;
  }
}

template <class SI, class SO, class LK, class T, int SEL, int NR>
static void dslash_go(hipStream_t st, const DslashArgs& a, int nprop) {
  int tiles = a.np * ((a.nb * a.g.Vbh + 255) / 256);
  dim3 grid(tiles, (a.nrhs + NR - 1) / NR, nprop);
  launch_timed((k_dslash<SI, SO, LK, T, SEL, NR>), grid, dim3(256), 0, st, a);
}

template <class SI, class SO, class LK, class T, int SEL>
static void dslash_nr(hipStream_t st, const DslashArgs& a, int nprop, int nr) {
  if (nr >= 4 && a.nrhs >= 4) dslash_go<SI, SO, LK, T, SEL, 4>(st, a, nprop);
  else if (nr >= 2 && a.nrhs >= 2) dslash_go<SI, SO, LK, T, SEL, 2>(st, a, nprop);
  else dslash_go<SI, SO, LK, T, SEL, 1>(st, a, nprop);
}

template <class SI, class SO, class LK, class T>
static void dslash_sel(hipStream_t st, const DslashArgs& a, int nprop, int sel, int nr) {
  if (sel == HOP_ALL) dslash_nr<SI, SO, LK, T, HOP_ALL>(st, a, nprop, nr);
  else if (sel == HOP_INTRA) dslash_nr<SI, SO, LK, T, HOP_INTRA>(st, a, nprop, nr);
  else dslash_nr<SI, SO, LK, T, HOP_CROSS>(st, a, nprop, nr);
}

// The kernel that stencil form v launches for these storages (as dslash_variant does)
template <class SI, class SO, class LK, class T>
static const void* variant_kernel(int v) {
  switch (v) {
    case 8: return reinterpret_cast<const void*>(&k_dslash_tile<SI, SO, LK, T, 1>);
    case 7: return reinterpret_cast<const void*>(&k_dslash_block<SI, SO, LK, T, 1>);
    case 1: return reinterpret_cast<const void*>(&k_dslash_split<SI, SO, LK, T, 1>);
    case 2: return reinterpret_cast<const void*>(&k_dslash<SI, SO, LK, T, HOP_ALL, 1, 4>);
    case 3: return reinterpret_cast<const void*>(&k_dslash_split<SI, SO, LK, T, 4>);
    case 4: return reinterpret_cast<const void*>(&k_dslash<SI, SO, LK, T, HOP_ALL, 1, 6>);
    case 5: return reinterpret_cast<const void*>(&k_dslash_split<SI, SO, LK, T, 6>);
    case 6: return reinterpret_cast<const void*>(&k_dslash_quad<SI, SO, LK, T, 2>);
    default: return reinterpret_cast<const void*>(&k_dslash<SI, SO, LK, T, HOP_ALL, 1, 1>);
  }
}

size_t dslash_variant_scratch(Prec in, Prec out, int v) {
  const void* f;
  if (in == P_F64) f = variant_kernel<StF64, StF64, LkF64, double>(v);
  else if (in == P_F32) f = variant_kernel<StF32, StF32, LkF32C12, float>(v);
  else if (out == P_BF16) f = variant_kernel<StBF16, StBF16, LkF32C12, float>(v);
  else f = variant_kernel<StBF16, StF32, LkF32C12, float>(v);
  hipFuncAttributes attr;
  if (hipFuncGetAttributes(&attr, f) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return attr.localSizeBytes;
}

void launch_dslash(hipStream_t st, const Geo& g, const void* const* links, int linkfmt, const FieldBatch& in,
                   const FieldBatch& out, const DslashParams& dp, int nr_pref) {
  DslashArgs a;
  a.g = g;
  for (int i = 0; i < MAXPROP; ++i) a.links[i] = i < in.nprop ? links[i] : nullptr;
  a.in = in.p;
  a.out = out.p;
  a.in_rhs_stride = units_per_field(in.prec, g.Vh);
  a.out_rhs_stride = units_per_field(out.prec, g.Vh);
  a.nrhs = in.nrhs;
  a.p0 = dp.p0;
  a.np = dp.np;
  a.blk0 = dp.blk0;
  a.nb = dp.nb;
  a.cdiag = dp.cdiag;
  a.chop = dp.chop;
  a.accumulate = dp.accumulate;
  a.xcd_map = dp.xcd_map;
  // an output larger than the 8 XCD L2 caches (8 x 4 MB) cannot be re-read from L2 by
  // the next kernel anyway: stream it past the cache
  a.nt_out = double(bytes_per_field(out.prec, g.Vh)) * out.nrhs * out.nprop > 32.0 * (1 << 20) ? 1 : 0;
  // the stencil forms exist for these storage pairs; any other pair runs the one-lane form
  const bool has_forms = (in.prec == P_F64 && out.prec == P_F64 && linkfmt == LK_F64) ||
                         (in.prec != P_F64 && linkfmt == LK_F32C12 &&
                          ((in.prec == P_F32 && out.prec == P_F32) || (in.prec == P_BF16 && out.prec != P_F64)));
  if (dp.variant > 0 && dp.sel == HOP_ALL && nr_pref <= 1 && has_forms) {
    if (in.prec == P_F64)
      dslash_variant<StF64, StF64, LkF64, double>(st, a, in.nprop, dp.variant);
    else if (in.prec == P_F32)
      dslash_variant<StF32, StF32, LkF32C12, float>(st, a, in.nprop, dp.variant);
    else if (out.prec == P_BF16)
      dslash_variant<StBF16, StBF16, LkF32C12, float>(st, a, in.nprop, dp.variant);
    else
      dslash_variant<StBF16, StF32, LkF32C12, float>(st, a, in.nprop, dp.variant);
    return;
  }
  if (in.prec == P_F64 && out.prec == P_F64 && linkfmt == LK_F64)
    dslash_sel<StF64, StF64, LkF64, double>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_F32 && out.prec == P_F32 && linkfmt == LK_F32C12)
    dslash_sel<StF32, StF32, LkF32C12, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_BF16 && out.prec == P_BF16 && linkfmt == LK_F32C12)
    dslash_sel<StBF16, StBF16, LkF32C12, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_BF16 && out.prec == P_F32 && linkfmt == LK_F32C12)
    dslash_sel<StBF16, StF32, LkF32C12, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_F32 && out.prec == P_BF16 && linkfmt == LK_F32C12)
    dslash_sel<StF32, StBF16, LkF32C12, float>(st, a, in.nprop, dp.sel, nr_pref);
  // FP32 18-real links (fields that are not SU(3)): the one-lane forms
  else if (in.prec == P_F32 && out.prec == P_F32 && linkfmt == LK_F32F18)
    dslash_sel<StF32, StF32, LkF32F18, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_BF16 && out.prec == P_BF16 && linkfmt == LK_F32F18)
    dslash_sel<StBF16, StBF16, LkF32F18, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_BF16 && out.prec == P_F32 && linkfmt == LK_F32F18)
    dslash_sel<StBF16, StF32, LkF32F18, float>(st, a, in.nprop, dp.sel, nr_pref);
  else if (in.prec == P_F32 && out.prec == P_BF16 && linkfmt == LK_F32F18)
    dslash_sel<StF32, StBF16, LkF32F18, float>(st, a, in.nprop, dp.sel, nr_pref);
}

// ----------------------------------------------------------------- layout conversion
// out (layout `to`) = in (layout `from`): the same fields in another block order.
// Parity is a property of the site, so only the index within the parity changes.
template <class S>
__global__ void k_permute(Geo from, Geo to, const typename S::unit* __restrict__ in, typename S::unit* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * to.Vh) return;
  const int p = t / to.Vh, s = t - p * to.Vh;
  SiteInfo si;
  site_info(to, p, s, si);
  int x[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) x[m] = si.B[m] * to.b[m] + si.l[m];
  int pf, sf;
  coords_to_internal(from, x, pf, sf);
  const size_t Vh = to.Vh, off = size_t(blockIdx.y) * 2 * S::NC * Vh;
#pragma unroll
  for (int k = 0; k < S::NC; ++k) out[off + (size_t(p) * S::NC + k) * Vh + s] = in[off + (size_t(pf) * S::NC + k) * Vh + sf];
}

void launch_permute(hipStream_t st, const Geo& from, const Geo& to, const FieldBatch& in, const FieldBatch& out) {
  dim3 grid((2 * to.Vh + 255) / 256, in.nprop * in.nrhs);
  if (in.prec == P_F64) hipLaunchKernelGGL(k_permute<StF64>, grid, dim3(256), 0, st, from, to, (const double2*)in.p, (double2*)out.p);
  else if (in.prec == P_F32) hipLaunchKernelGGL(k_permute<StF32>, grid, dim3(256), 0, st, from, to, (const float4*)in.p, (float4*)out.p);
  else hipLaunchKernelGGL(k_permute<StBF16>, grid, dim3(256), 0, st, from, to, (const uint4*)in.p, (uint4*)out.p);
}

template <class S, class T>
__global__ void k_pack(Geo g, const double* __restrict__ src, typename S::unit* __restrict__ dst, int V) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int rhs = blockIdx.y;
  int p, s;
  lex_to_internal(g, lex, p, s);
  const double* q = src + (size_t(rhs) * V + lex) * 24;
  Spinor<T> sp;
#pragma unroll
  for (int k = 0; k < 12; ++k) sp.v[k / 3][k % 3] = {T(q[2 * k]), T(q[2 * k + 1])};
  S::store(dst + size_t(rhs) * 2 * S::NC * g.Vh + size_t(p) * S::NC * g.Vh, g.Vh, s, sp);
}

template <class S, class T>
__global__ void k_unpack(Geo g, const typename S::unit* __restrict__ src, double* __restrict__ dst, int V) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int rhs = blockIdx.y;
  int p, s;
  lex_to_internal(g, lex, p, s);
  Spinor<T> sp;
  S::load(src + size_t(rhs) * 2 * S::NC * g.Vh + size_t(p) * S::NC * g.Vh, g.Vh, s, sp);
  double* q = dst + (size_t(rhs) * V + lex) * 24;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    q[2 * k] = double(sp.v[k / 3][k % 3].re);
    q[2 * k + 1] = double(sp.v[k / 3][k % 3].im);
  }
}

void launch_pack(hipStream_t st, const Geo& g, const double* src, const FieldBatch& dst) {
  int V = 2 * g.Vh;
  dim3 grid((V + 255) / 256, dst.nprop * dst.nrhs);
  if (dst.prec == P_F64) hipLaunchKernelGGL((k_pack<StF64, double>), grid, dim3(256), 0, st, g, src, (double2*)dst.p, V);
  else if (dst.prec == P_F32) hipLaunchKernelGGL((k_pack<StF32, float>), grid, dim3(256), 0, st, g, src, (float4*)dst.p, V);
  else hipLaunchKernelGGL((k_pack<StBF16, float>), grid, dim3(256), 0, st, g, src, (uint4*)dst.p, V);
}

void launch_unpack(hipStream_t st, const Geo& g, const FieldBatch& src, double* dst) {
  int V = 2 * g.Vh;
  dim3 grid((V + 255) / 256, src.nprop * src.nrhs);
  if (src.prec == P_F64) hipLaunchKernelGGL((k_unpack<StF64, double>), grid, dim3(256), 0, st, g, (const double2*)src.p, dst, V);
  else if (src.prec == P_F32) hipLaunchKernelGGL((k_unpack<StF32, float>), grid, dim3(256), 0, st, g, (const float4*)src.p, dst, V);
  else hipLaunchKernelGGL((k_unpack<StBF16, float>), grid, dim3(256), 0, st, g, (const uint4*)src.p, dst, V);
}

__global__ void k_pack_links(Geo g, const double* __restrict__ U, void* __restrict__ dst, int V, int fmt) {
  int lex = blockIdx.x * blockDim.x + threadIdx.x;
  if (lex >= V) return;
  int p, s;
  lex_to_internal(g, lex, p, s);
  const size_t Vh = g.Vh;
  for (int mu = 0; mu < 4; ++mu) {
    const double* q = U + (size_t(lex) * 4 + mu) * 18;
    if (fmt == LK_F64) {
      double2* d = reinterpret_cast<double2*>(dst) + size_t(p * 4 + mu) * 9 * Vh;
      for (int k = 0; k < 9; ++k) d[k * Vh + s] = make_double2(q[2 * k], q[2 * k + 1]);
    } else {
      float4* d = reinterpret_cast<float4*>(dst) + size_t(p * 4 + mu) * 3 * Vh;
      for (int k = 0; k < 3; ++k)
        d[k * Vh + s] = make_float4(float(q[4 * k]), float(q[4 * k + 1]), float(q[4 * k + 2]), float(q[4 * k + 3]));
    }
  }
}

void launch_pack_links(hipStream_t st, const Geo& g, const double* U, void* dst, int linkfmt) {
  int V = 2 * g.Vh;
  hipLaunchKernelGGL(k_pack_links, dim3((V + 255) / 256), dim3(256), 0, st, g, U, dst, V, linkfmt);
}

// Deviation of each link from SU(3): max(|U U^+ - 1|_max, |det U - 1|).
// Links U(x, mu) with x_mu mod ob_mu = ob_mu - 1 leave x's outer block: set to zero.
__global__ void k_cut_links(Geo g, void* __restrict__ links, int fmt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  const int p = t / g.Vh, s = t - p * g.Vh;
  SiteInfo si;
  site_info(g, p, s, si);
  const size_t Vh = g.Vh;
  for (int mu = 0; mu < 4; ++mu) {
    const int x = si.B[mu] * g.b[mu] + si.l[mu];
    if (x % g.ob[mu] != g.ob[mu] - 1) continue;
    if (fmt == LK_F64) {
      double2* d = reinterpret_cast<double2*>(links) + size_t(p * 4 + mu) * 9 * Vh;
      for (int k = 0; k < 9; ++k) d[k * Vh + s] = make_double2(0.0, 0.0);
    } else {
      float4* d = reinterpret_cast<float4*>(links) + size_t(p * 4 + mu) * 3 * Vh;
      for (int k = 0; k < 3; ++k) d[k * Vh + s] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

void launch_cut_links(hipStream_t st, const Geo& g, void* links, int linkfmt) {
  hipLaunchKernelGGL(k_cut_links, dim3((2 * g.Vh + 255) / 256), dim3(256), 0, st, g, links, linkfmt);
}

__global__ void k_links_f64_to_f18(Geo g, const double2* __restrict__ src, float4* __restrict__ dst) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  const int p = t / g.Vh, s = t - p * g.Vh;
  const size_t Vh = g.Vh;
  for (int mu = 0; mu < 4; ++mu) {
    const double2* a = src + size_t(p * 4 + mu) * LkF64::NC * Vh;
    float4* d = dst + size_t(p * 4 + mu) * LkF32F18::NC * Vh;
    for (int k = 0; k < 5; ++k) {
      const double2 x = a[(2 * k) * Vh + s];
      const double2 y = 2 * k + 1 < 9 ? a[(2 * k + 1) * Vh + s] : make_double2(0.0, 0.0);
      d[k * Vh + s] = make_float4(float(x.x), float(x.y), float(y.x), float(y.y));
    }
  }
}
void launch_links_f64_to_f18(hipStream_t st, const Geo& g, const void* f64, void* f18) {
  hipLaunchKernelGGL(k_links_f64_to_f18, dim3((2 * g.Vh + 255) / 256), dim3(256), 0, st, g,
                     (const double2*)f64, (float4*)f18);
}

// max that keeps a NaN (fmax drops it), so a link holding NaN or Inf marks the field
__device__ __forceinline__ double nan_max(double a, double b) { return (b > a || b != b) ? b : a; }

__global__ void k_unitarity(const double* __restrict__ U, int nlinks, double* __restrict__ partial) {
  __shared__ double sm[256];
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  double dev = 0.0;
  for (int l = t; l < nlinks; l += gridDim.x * blockDim.x) {
    const double* q = U + size_t(l) * 18;
    cx<double> m[3][3];
    for (int k = 0; k < 9; ++k) m[k / 3][k % 3] = {q[2 * k], q[2 * k + 1]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cx<double> a = cjmul(m[j][0], m[i][0]) + cjmul(m[j][1], m[i][1]) + cjmul(m[j][2], m[i][2]);
        double re = a.re - (i == j ? 1.0 : 0.0);
        dev = nan_max(dev, nan_max(fabs(re), fabs(a.im)));
      }
    cx<double> det = cmul(m[0][0], cmul(m[1][1], m[2][2]) - cmul(m[1][2], m[2][1])) -
                     cmul(m[0][1], cmul(m[1][0], m[2][2]) - cmul(m[1][2], m[2][0])) +
                     cmul(m[0][2], cmul(m[1][0], m[2][1]) - cmul(m[1][1], m[2][0]));
    dev = nan_max(dev, nan_max(fabs(det.re - 1.0), fabs(det.im)));
  }
  sm[threadIdx.x] = dev;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sm[threadIdx.x] = nan_max(sm[threadIdx.x], sm[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sm[0];
}

void launch_unitarity(hipStream_t st, const Geo& g, const double* U, double* partial, int nwg) {
  hipLaunchKernelGGL(k_unitarity, dim3(nwg), dim3(256), 0, st, U, 8 * g.Vh, partial);
}

// ----------------------------------------------------------------- projector P
// (1 + s gamma_mu) psi for s = +1 / -1, built from the two projected spin rows.
template <class T> __device__ __forceinline__ void one_pm_gamma(int mu, int s, const Spinor<T>& p, Spinor<T>& o) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cx<T> h0, h1;
    if (s > 0) {  // 1 + gamma_mu
      switch (mu) {
        case 0: h0 = p.v[0][a] - p.v[2][a]; h1 = p.v[1][a] - p.v[3][a];
                o.v[2][a] = -h0; o.v[3][a] = -h1; break;
        case 1: h0 = p.v[0][a] + times_mi(p.v[3][a]); h1 = p.v[1][a] + times_mi(p.v[2][a]);
                o.v[2][a] = times_i(h1); o.v[3][a] = times_i(h0); break;
        case 2: h0 = p.v[0][a] - p.v[3][a]; h1 = p.v[1][a] + p.v[2][a];
                o.v[2][a] = h1; o.v[3][a] = -h0; break;
        default: h0 = p.v[0][a] + times_mi(p.v[2][a]); h1 = p.v[1][a] + times_i(p.v[3][a]);
                o.v[2][a] = times_i(h0); o.v[3][a] = times_mi(h1); break;
      }
    } else {  // 1 - gamma_mu
      switch (mu) {
        case 0: h0 = p.v[0][a] + p.v[2][a]; h1 = p.v[1][a] + p.v[3][a];
                o.v[2][a] = h0; o.v[3][a] = h1; break;
        case 1: h0 = p.v[0][a] + times_i(p.v[3][a]); h1 = p.v[1][a] + times_i(p.v[2][a]);
                o.v[2][a] = times_mi(h1); o.v[3][a] = times_mi(h0); break;
        case 2: h0 = p.v[0][a] + p.v[3][a]; h1 = p.v[1][a] - p.v[2][a];
                o.v[2][a] = -h1; o.v[3][a] = h0; break;
        default: h0 = p.v[0][a] + times_i(p.v[2][a]); h1 = p.v[1][a] + times_mi(p.v[3][a]);
                o.v[2][a] = times_mi(h0); o.v[3][a] = times_i(h1); break;
      }
    }
    o.v[0][a] = h0;
    o.v[1][a] = h1;
  }
}

template <class S, class T>
__global__ void k_project(Geo g, const typename S::unit* __restrict__ in, typename S::unit* __restrict__ out) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * g.Vh) return;
  int p = t / g.Vh, s = t - p * g.Vh;
  size_t off = size_t(blockIdx.y) * 2 * S::NC * g.Vh + size_t(p) * S::NC * g.Vh;
  SiteInfo si;
  site_info(g, p, s, si);
  Spinor<T> o;
  zero(o);
  if (si.colour == 0) {
    int nout = 0, mu1 = 0, dir1 = 0;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      // with outer blocks, a hop across an outer face is not part of the operator
      const int x = si.B[mu] * g.b[mu] + si.l[mu];
      const bool cut_f = g.ob[mu] && x % g.ob[mu] == g.ob[mu] - 1, cut_b = g.ob[mu] && x % g.ob[mu] == 0;
      if (si.l[mu] == g.b[mu] - 1 && !cut_f) { ++nout; mu1 = mu; dir1 = +1; }
      if (si.l[mu] == 0 && !cut_b) { ++nout; mu1 = mu; dir1 = -1; }
    }
    if (nout > 0) {
      Spinor<T> x;
      S::load(in + off, g.Vh, s, x);
      if (nout >= 2) {
        o = x;
      } else {
        // outside neighbour at y + mu -> (1 + gamma_mu)/2 ; at y - mu -> (1 - gamma_mu)/2
        one_pm_gamma(mu1, dir1, x, o);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) o.v[a][c] = scale(T(0.5), o.v[a][c]);
      }
    }
  }
  S::store(out + off, g.Vh, s, o);
}

void launch_project(hipStream_t st, const Geo& g, const FieldBatch& in, const FieldBatch& out) {
  dim3 grid((2 * g.Vh + 255) / 256, in.nprop * in.nrhs);
  if (in.prec == P_F64) hipLaunchKernelGGL((k_project<StF64, double>), grid, dim3(256), 0, st, g, (const double2*)in.p, (double2*)out.p);
  else if (in.prec == P_F32) hipLaunchKernelGGL((k_project<StF32, float>), grid, dim3(256), 0, st, g, (const float4*)in.p, (float4*)out.p);
  else hipLaunchKernelGGL((k_project<StBF16, float>), grid, dim3(256), 0, st, g, (const uint4*)in.p, (uint4*)out.p);
}

}  // namespace psms
