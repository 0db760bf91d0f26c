// Gauge-covariant linear network (learned preconditioner): layer forward and
// adjoint, weight gradients, Adam, and the counter-based Gaussian generator that
// draws the training right-hand sides.
//
// Layer: Psi_c(x) = sum_t sum_c' W[t][c][c'] (T_t Phi_c')(x), T_0 = 1,
// T_{1+2mu} Phi(x) = U(x,mu) Phi(x+mu), T_{2+2mu} Phi(x) = U(x-mu,mu)^+ Phi(x-mu)
// (fermion boundary sign across the time boundary), W[t][c][c'] a complex 4x4
// spin matrix. The adjoint (input gradient) is the same kernel with
// W'[opp(t)][c'][c] = W[t][c][c']^+.
//
// A workgroup owns NS = 64 sites. For each of the 9 transports it stages the
// transported inputs of its sites in LDS (one complex plane per spin-colour
// component), then every (site, output channel) task mixes them with the 4x4
// spin matrices held in LDS. Activations are stored as F32 spinor fields
// ([batch][channel][parity][6 float4 planes][Vh]).
#include <algorithm>

#include "kernels.h"

namespace psms {

constexpr int NET_NS = 64;
constexpr int NET_MAXC = 8;

__device__ __forceinline__ int net_opp(int t) { return t == 0 ? 0 : ((t & 1) ? t + 1 : t - 1); }

// T_t Phi at site (p, s) of one F32 field.
__device__ __forceinline__ void net_transport(const Geo& g, const float4* __restrict__ lk, const float4* __restrict__ phi,
                                              int p, int s, const SiteInfo& si, int t, Spinor<float>& o) {
  const size_t Vh = g.Vh;
  if (t == 0) {
    StF32::load(phi + size_t(p) * 6 * Vh, Vh, s, o);
    return;
  }
  const int mu = (t - 1) >> 1;
  const bool fwd = ((t - 1) & 1) == 0;
  Nbr n = neighbour(g, si, mu, fwd ? +1 : -1);
  SU3<float> U;
  if (fwd) LkF32C12::load(lk + size_t(p * 4 + mu) * 3 * Vh, Vh, s, U);
  else LkF32C12::load(lk + size_t((1 - p) * 4 + mu) * 3 * Vh, Vh, n.s, U);
  Spinor<float> v;
  StF32::load(phi + size_t(1 - p) * 6 * Vh, Vh, n.s, v);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp) {
    cx<float> w[3];
    if (fwd) su3_mul_sum(U, v.v[sp], w);
    else su3_dag_mul_sum(U, v.v[sp], w);
#pragma unroll
    for (int a = 0; a < 3; ++a) o.v[sp][a] = scale(n.sign, w[a]);
  }
}

struct NetLayerArgs {
  Geo g;
  const float4* links;
  const float4* in;   // [batch][cin][field]
  float4* out;        // [batch][cout][field]
  const float2* W;    // forward layer weights [9][cout_f][cin_f][4][4]
  int cin, cout;      // channels of this launch
  int cin_f, cout_f;  // channels of the forward layer
  int adj;
};

__global__ void __launch_bounds__(256) k_net_layer(NetLayerArgs a) {
  __shared__ cx<float> tp[NET_MAXC][12][NET_NS];          // transported inputs of the tile
  __shared__ cx<float> wl[NET_MAXC][NET_MAXC][16];         // spin matrices for this transport
  const Geo& g = a.g;
  const size_t Vh = g.Vh, fsz = size_t(2) * 6 * Vh;
  const int site0 = blockIdx.x * NET_NS;
  const int b = blockIdx.y;
  const float4* in = a.in + size_t(b) * a.cin * fsz;
  float4* out = a.out + size_t(b) * a.cout * fsz;
  const int ntask = NET_NS * a.cout;
  // each thread keeps the accumulators of up to two (site, output channel) tasks
  Spinor<float> acc[2];
  zero(acc[0]);
  zero(acc[1]);
  for (int u = 0; u < 9; ++u) {
    // stage transported inputs and the weights of this transport
    for (int task = threadIdx.x; task < NET_NS * a.cin; task += blockDim.x) {
      const int l = task % NET_NS, ci = task / NET_NS;
      const int site = site0 + l;
      Spinor<float> v;
      if (site < 2 * g.Vh) {
        const int p = site / g.Vh, s = site - p * g.Vh;
        SiteInfo si;
        site_info(g, p, s, si);
        net_transport(g, a.links, in + size_t(ci) * fsz, p, s, si, u, v);
      } else {
        zero(v);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) tp[ci][k][l] = v.v[k / 3][k % 3];
    }
    const int t = a.adj ? net_opp(u) : u;
    for (int e = threadIdx.x; e < a.cout * a.cin * 16; e += blockDim.x) {
      const int co = e / (a.cin * 16), ci = (e / 16) % a.cin, ss = e % 16;
      const int s1 = ss / 4, s2 = ss % 4;
      float2 w;
      if (!a.adj) {
        w = a.W[((size_t(t) * a.cout_f + co) * a.cin_f + ci) * 16 + s1 * 4 + s2];
      } else {  // W[t][ci][co]^+ : element (s1, s2) = conj(W[t][ci][co](s2, s1))
        w = a.W[((size_t(t) * a.cout_f + ci) * a.cin_f + co) * 16 + s2 * 4 + s1];
        w.y = -w.y;
      }
      wl[co][ci][ss] = {w.x, w.y};
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int task = threadIdx.x + j * blockDim.x;
      if (task < ntask) {
        const int l = task % NET_NS, co = task / NET_NS;
        for (int ci = 0; ci < a.cin; ++ci) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            cx<float> x0 = tp[ci][0 * 3 + c][l], x1 = tp[ci][1 * 3 + c][l], x2 = tp[ci][2 * 3 + c][l], x3 = tp[ci][3 * 3 + c][l];
#pragma unroll
            for (int s1 = 0; s1 < 4; ++s1) {
              acc[j].v[s1][c] = acc[j].v[s1][c] + cmul(wl[co][ci][s1 * 4 + 0], x0) + cmul(wl[co][ci][s1 * 4 + 1], x1) +
                                cmul(wl[co][ci][s1 * 4 + 2], x2) + cmul(wl[co][ci][s1 * 4 + 3], x3);
            }
          }
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int task = threadIdx.x + j * blockDim.x;
    if (task < ntask) {
      const int l = task % NET_NS, co = task / NET_NS;
      const int site = site0 + l;
      if (site < 2 * g.Vh) {
        const int p = site / g.Vh, s = site - p * g.Vh;
        StF32::store(out + size_t(co) * fsz + size_t(p) * 6 * Vh, Vh, s, acc[j]);
      }
    }
  }
}

void launch_net_layer(hipStream_t st, const Geo& g, const void* links, const void* in, void* out, const float2* W, int cin_f,
                      int cout_f, int adj, int batch) {
  NetLayerArgs a;
  a.g = g;
  a.links = (const float4*)links;
  a.in = (const float4*)in;
  a.out = (float4*)out;
  a.W = W;
  a.cin_f = cin_f;
  a.cout_f = cout_f;
  a.adj = adj;
  a.cin = adj ? cout_f : cin_f;
  a.cout = adj ? cin_f : cout_f;
  dim3 grid((2 * g.Vh + NET_NS - 1) / NET_NS, batch);
  hipLaunchKernelGGL(k_net_layer, grid, dim3(256), 0, st, a);
}

// ---------------------------------------------------------------- MFMA form of the layer
// The channel mixing of a tile is one real GEMM Y[M x N] = A[M x K] B[K x N] on the
// matrix cores (bf16 inputs, FP32 accumulation, v_mfma_f32_32x32x8_bf16):
//   rows  m = (c, s, re/im)              M = 8 c_out  (padded to a multiple of 32)
//   cols  n = (site, colour)             N = 3 * 64
//   depth k = (t, c', s', re/im)         K = 72 c_in
// with the complex 4x4 spin matrices embedded as [[Wr, -Wi], [Wi, Wr]]. A is packed
// once per weight update into per-lane fragments; B (the transported inputs of one
// direction t) is staged in LDS as bf16, k fastest; Y goes through LDS so that the
// output spinors are written with coalesced stores.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ short to_bf16(float f) { return short(f32_to_bf16(f)); }

// Apack[(mb * ksteps + kb) * 64 + lane] holds A[mb*32 + lane%32][kb*8 + (lane/32)*4 + q], q = 0..3.
__global__ void k_net_pack(const float2* __restrict__ W, int cin_f, int cout_f, int adj, uint2* __restrict__ Apack) {
  const int cin = adj ? cout_f : cin_f, cout = adj ? cin_f : cout_f;
  const int M = 8 * cout, mblk = (M + 31) / 32, ksteps = 9 * cin;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= mblk * ksteps * 64) return;
  const int lane = idx & 63, kb = (idx >> 6) % ksteps, mb = (idx >> 6) / ksteps;
  const int m = mb * 32 + (lane & 31);
  short v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = kb * 8 + (lane >> 5) * 4 + q;
    float a = 0.f;
    if (m < M) {
      const int ri = m & 1, s = (m >> 1) & 3, co = m >> 3;
      const int rj = k & 1, s2 = (k >> 1) & 3, ci = (k >> 3) % cin, u = (k >> 3) / cin;
      float2 w;
      if (!adj) {
        w = W[((size_t(u) * cout_f + co) * cin_f + ci) * 16 + s * 4 + s2];
      } else {
        w = W[((size_t(net_opp(u)) * cout_f + ci) * cin_f + co) * 16 + s2 * 4 + s];
        w.y = -w.y;
      }
      a = (ri == rj) ? w.x : (ri == 0 ? -w.y : w.y);
    }
    v[q] = to_bf16(a);
  }
  Apack[idx] = make_uint2(uint32_t(uint16_t(v[0])) | (uint32_t(uint16_t(v[1])) << 16),
                          uint32_t(uint16_t(v[2])) | (uint32_t(uint16_t(v[3])) << 16));
}

size_t net_pack_units(int cin_f, int cout_f, int adj) {
  const int cin = adj ? cout_f : cin_f, cout = adj ? cin_f : cout_f;
  return size_t((8 * cout + 31) / 32) * 9 * cin * 64;
}

void launch_net_pack(hipStream_t st, const float2* W, int cin_f, int cout_f, int adj, uint2* Apack) {
  const size_t n = net_pack_units(cin_f, cout_f, adj);
  hipLaunchKernelGGL(k_net_pack, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, W, cin_f, cout_f, adj, Apack);
}

constexpr int NET_KPAD = 8 * NET_MAXC + 4;   // bf16 row stride of the staged B tile (breaks bank aliasing)
constexpr int NET_CPAD = 3 * NET_NS + 4;     // float row stride of the staged output tile

struct NetMfmaArgs {
  Geo g;
  const float4* links;
  const float4* in;
  float4* out;
  const uint2* A;
  int cin, cout;  // channels of this launch
};

template <int W>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W))) k_net_layer_mfma(NetMfmaArgs a) {
  // the staged input tile (bf16) and the output tile (FP32) share one LDS buffer:
  // the output is written only after the last MFMA has read the inputs
  constexpr size_t kB = sizeof(short) * 3 * NET_NS * NET_KPAD, kC = sizeof(float) * 8 * NET_MAXC * NET_CPAD;
  __shared__ float4 lds_raw[(kB > kC ? kB : kC) / 16];
  short(*Bs)[NET_KPAD] = reinterpret_cast<short(*)[NET_KPAD]>(lds_raw);
  float(*Cs)[NET_CPAD] = reinterpret_cast<float(*)[NET_CPAD]>(lds_raw);
  const Geo& g = a.g;
  const size_t Vh = g.Vh, fsz = size_t(2) * 6 * Vh;
  const int site0 = blockIdx.x * NET_NS;
  const int b = blockIdx.y;
  const float4* in = a.in + size_t(b) * a.cin * fsz;
  float4* out = a.out + size_t(b) * a.cout * fsz;
  const int M = 8 * a.cout, mblk = (M + 31) / 32, ksteps = 9 * a.cin, nblk = 3 * NET_NS / 32;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // output blocks: wave w takes blk = w + 4 i, i.e. (mb, nb) = (blk % mblk, blk / mblk);
  // mblk divides 4, so all of a wave's blocks share mb and one A fragment per k-step
  const int mbw = wave % mblk;
  f32x16 acc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[i][v] = 0.f;
  // staging: thread -> one site (l) and the channels cg, cg + 4; its neighbours and
  // boundary signs are computed once, each link is loaded once for both channels
  static_assert(NET_NS == 64 && NET_MAXC == 8, "staging assumes 64 sites and at most 8 channels");
  static_assert(4 % ((8 * NET_MAXC + 31) / 32) == 0, "the row blocks of the output divide the 4 waves");
  const int l = threadIdx.x & 63, cg = threadIdx.x >> 6;
  const int site = site0 + l;
  const bool valid = site < 2 * g.Vh;
  int p = 0, s = 0, nsite[8];
  float nsign[8];
  if (valid) {
    p = site / g.Vh;
    s = site - p * g.Vh;
    SiteInfo si;
    site_info(g, p, s, si);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      Nbr n = neighbour(g, si, k >> 1, (k & 1) ? -1 : +1);
      nsite[k] = n.s;
      nsign[k] = n.sign;
    }
  }
  // software pipeline: the link and spinors of direction t + 1 are loaded while the
  // matrix cores work on direction t
  SU3<float> U;
  Spinor<float> xs[2];
  auto fetch = [&](int t) {
    if (!valid) return;
    int ps = p, ss = s;
    if (t > 0) {
      const int mu = (t - 1) >> 1;
      const bool fwd = ((t - 1) & 1) == 0;
      ps = 1 - p;
      ss = nsite[t - 1];
      if (fwd) LkF32C12::load(a.links + size_t(p * 4 + mu) * 3 * Vh, Vh, s, U);
      else LkF32C12::load(a.links + size_t((1 - p) * 4 + mu) * 3 * Vh, Vh, ss, U);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (cg + 4 * h < a.cin) StF32::load(in + size_t(cg + 4 * h) * fsz + size_t(ps) * 6 * Vh, Vh, ss, xs[h]);
  };
  fetch(0);
  for (int t = 0; t < 9; ++t) {
    // the A fragments of direction t, requested before the staging hides their latency
    uint2 af[NET_MAXC];
#pragma unroll
    for (int kk = 0; kk < NET_MAXC; ++kk)
      if (kk < a.cin) af[kk] = a.A[(size_t(mbw) * ksteps + t * a.cin + kk) * 64 + lane];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int ci = cg + 4 * h;
      if (ci < a.cin) {
        Spinor<float> v;
        if (valid) {
          const Spinor<float>& x = xs[h];
          if (t == 0) {
            v = x;
          } else {
            const bool fwd = ((t - 1) & 1) == 0;
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
              cx<float> w[3];
              if (fwd) su3_mul_sum(U, x.v[sp], w);
              else su3_dag_mul_sum(U, x.v[sp], w);
#pragma unroll
              for (int c = 0; c < 3; ++c) v.v[sp][c] = scale(nsign[t - 1], w[c]);
            }
          }
        } else {
          zero(v);
        }
        // the 8 bf16 of one colour (4 spins x re/im) are contiguous: two 8-byte stores
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          // the matrix cores' operands round with gfx950's one-instruction conversion (its
          // last-bit choices on some inputs do not matter at bf16 precision)
          uint32_t w[4];
#pragma unroll
          for (int sp = 0; sp < 4; ++sp) w[sp] = bf16_pack2(v.v[sp][c].re, v.v[sp][c].im);
          uint2* dst = reinterpret_cast<uint2*>(&Bs[l * 3 + c][ci * 8]);
          dst[0] = make_uint2(w[0], w[1]);
          dst[1] = make_uint2(w[2], w[3]);
        }
      }
    }
    __syncthreads();
    if (t < 8) fetch(t + 1);
#pragma unroll
    for (int kk = 0; kk < NET_MAXC; ++kk) {
      if (kk < a.cin) {
        const uint2 au = af[kk];
        bf16x4 av;
        av[0] = short(au.x & 0xffffu); av[1] = short(au.x >> 16); av[2] = short(au.y & 0xffffu); av[3] = short(au.y >> 16);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const int blk = wave + 4 * i;
          if (blk < mblk * nblk) {
            const int nb = blk / mblk;
            const short* bp = &Bs[nb * 32 + (lane & 31)][kk * 8 + (lane >> 5) * 4];
            bf16x4 bv;
            bv[0] = bp[0]; bv[1] = bp[1]; bv[2] = bp[2]; bv[3] = bp[3];
            acc[i] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc[i], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  // accumulators -> LDS: lane, register v -> row (v/4)*8 + (lane/32)*4 + v%4, column lane%32
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int blk = wave + 4 * i;
    if (blk < mblk * nblk) {
      const int mb = blk % mblk, nb = blk / mblk;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = mb * 32 + (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3);
        if (row < M) Cs[row][nb * 32 + (lane & 31)] = acc[i][v];
      }
    }
  }
  __syncthreads();
  for (int task = threadIdx.x; task < NET_NS * a.cout; task += blockDim.x) {
    const int l = task % NET_NS, co = task / NET_NS;
    const int site = site0 + l;
    if (site < 2 * g.Vh) {
      Spinor<float> o;
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int c = 0; c < 3; ++c) o.v[sp][c] = {Cs[(co * 4 + sp) * 2][l * 3 + c], Cs[(co * 4 + sp) * 2 + 1][l * 3 + c]};
      const int p = site / g.Vh, s = site - p * g.Vh;
      StF32::store(out + size_t(co) * fsz + size_t(p) * 6 * Vh, Vh, s, o);
    }
  }
}

void launch_net_layer_mfma(hipStream_t st, const Geo& g, const void* links, const void* in, void* out, const uint2* Apack,
                           int cin_f, int cout_f, int adj, int batch) {
  NetMfmaArgs a;
  a.g = g;
  a.links = (const float4*)links;
  a.in = (const float4*)in;
  a.out = (float4*)out;
  a.A = Apack;
  a.cin = adj ? cout_f : cin_f;
  a.cout = adj ? cin_f : cout_f;
  dim3 grid((2 * g.Vh + NET_NS - 1) / NET_NS, batch);
  // Two waves per SIMD (no register limit): with the A fragments of a direction held in
  // registers, a form forced to three waves per SIMD spills 152 B per lane and takes
  // 4.45 ms per application at 16^4 x 8 fields against 3.07 ms. (A double-buffered
  // staged tile, staging direction t + 1 while the matrix cores take t, measured 3.13 ms.)
  hipLaunchKernelGGL((k_net_layer_mfma<1>), grid, dim3(256), 0, st, a);
}

// ---------------------------------------------------------------- weight gradient
// partial[w][t][co][ci][s1][s2] = sum over the tile's sites and colours of
// G_co(x)[s1,a] conj((T_t Phi_ci)(x)[s2,a]); w runs over (batch, tile).
struct NetGradArgs {
  Geo g;
  const float4* links;
  const float4* phi;  // forward input [batch][cin][field]
  const float4* G;    // gradient w.r.t. forward output [batch][cout][field]
  float2* partial;
  int cin, cout;
};

constexpr int NET_GS = 32;  // sites per workgroup of the gradient kernel

__global__ void __launch_bounds__(256) k_net_wgrad(NetGradArgs a) {
  __shared__ cx<float> gt[NET_MAXC][12][NET_GS];
  __shared__ cx<float> tp[NET_MAXC][12][NET_GS];
  const Geo& g = a.g;
  const size_t Vh = g.Vh, fsz = size_t(2) * 6 * Vh;
  const int b = blockIdx.y;
  const float4* phi = a.phi + size_t(b) * a.cin * fsz;
  const float4* G = a.G + size_t(b) * a.cout * fsz;
  const size_t wg = size_t(b) * gridDim.x + blockIdx.x;
  const int nent = a.cout * a.cin * 16;
  const int ntile = (2 * g.Vh + NET_GS - 1) / NET_GS;
  // accumulators of this thread's entries (e = threadIdx.x + 256 j), all transports
  cx<float> acc[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[t][j] = {0.f, 0.f};
  for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int site0 = tile * NET_GS;
    __syncthreads();
    for (int task = threadIdx.x; task < NET_GS * a.cout; task += blockDim.x) {
      const int l = task % NET_GS, co = task / NET_GS;
      const int site = site0 + l;
      Spinor<float> v;
      if (site < 2 * g.Vh) {
        const int p = site / g.Vh, s = site - p * g.Vh;
        StF32::load(G + size_t(co) * fsz + size_t(p) * 6 * Vh, Vh, s, v);
      } else {
        zero(v);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) gt[co][k][l] = v.v[k / 3][k % 3];
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      __syncthreads();
      for (int task = threadIdx.x; task < NET_GS * a.cin; task += blockDim.x) {
        const int l = task % NET_GS, ci = task / NET_GS;
        const int site = site0 + l;
        Spinor<float> v;
        if (site < 2 * g.Vh) {
          const int p = site / g.Vh, s = site - p * g.Vh;
          SiteInfo si;
          site_info(g, p, s, si);
          net_transport(g, a.links, phi + size_t(ci) * fsz, p, s, si, t, v);
        } else {
          zero(v);
        }
#pragma unroll
        for (int k = 0; k < 12; ++k) tp[ci][k][l] = v.v[k / 3][k % 3];
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int e = threadIdx.x + j * 256;
        if (e < nent) {
          const int co = e / (a.cin * 16), ci = (e / 16) % a.cin, s1 = (e % 16) / 4, s2 = e % 4;
          cx<float> sum = {0.f, 0.f};
          for (int l = 0; l < NET_GS; ++l) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sum = sum + cjmul(tp[ci][s2 * 3 + c][l], gt[co][s1 * 3 + c][l]);
          }
          acc[t][j] = acc[t][j] + sum;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = threadIdx.x + j * 256;
      if (e < nent) a.partial[(wg * 9 + t) * nent + e] = make_float2(acc[t][j].re, acc[t][j].im);
    }
}

// out[j] = sum_w partial[w][j] in double, fixed order
__global__ void k_net_reduce(const float2* __restrict__ partial, int nw, int n, double2* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double re = 0, im = 0;
  for (int w = 0; w < nw; ++w) {
    float2 v = partial[size_t(w) * n + j];
    re += v.x;
    im += v.y;
  }
  out[j] = make_double2(re, im);
}

constexpr int NET_GWG = 256;  // workgroups per batch entry in the gradient kernel
int net_wgrad_partials(const Geo& g, int batch) { return std::min(NET_GWG, (2 * g.Vh + NET_GS - 1) / NET_GS) * batch; }

void launch_net_wgrad(hipStream_t st, const Geo& g, const void* links, const void* phi, const void* G, int cin, int cout,
                      int batch, float2* partial, double2* grad_out) {
  NetGradArgs a;
  a.g = g;
  a.links = (const float4*)links;
  a.phi = (const float4*)phi;
  a.G = (const float4*)G;
  a.partial = partial;
  a.cin = cin;
  a.cout = cout;
  dim3 grid(std::min(NET_GWG, (2 * g.Vh + NET_GS - 1) / NET_GS), batch);
  hipLaunchKernelGGL(k_net_wgrad, grid, dim3(256), 0, st, a);
  const int n = 9 * cout * cin * 16;
  hipLaunchKernelGGL(k_net_reduce, dim3((n + 255) / 256), dim3(256), 0, st, partial, int(grid.x * grid.y), n, grad_out);
}

// ---------------------------------------------------------------- Adam (real view of the complex weights)
// g_real = 2 * dL/dconj(W) (re, im), decoupled from the FP32 master weights.
__global__ void k_adam(float* __restrict__ w, const double* __restrict__ grad, float* __restrict__ m, float* __restrict__ v, int n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gr = float(2.0 * grad[i]);
  const float mi = b1 * m[i] + (1.f - b1) * gr;
  const float vi = b2 * v[i] + (1.f - b2) * gr * gr;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_adam(hipStream_t st, float* w, const double* grad, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                 int step) {
  const float c1 = 1.f - powf(b1, float(step)), c2 = 1.f - powf(b2, float(step));
  hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, grad, m, v, n, lr, b1, b2, eps, c1, c2);
}

// ---------------------------------------------------------------- Gaussian fields (Philox4x32-10 + Box-Muller)
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xorshift bijection with the published multipliers and Weyl keys.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += W0;
    k.y += W1;
  }
  return c;
}

// Fills nfield F64 boundary-layout fields with complex Gaussians, density exp(-|z|^2)
// (real and imaginary parts N(0, 1/2)); element i of field f uses counter (i, f, stream).
__global__ void k_gaussian(double* __restrict__ out, size_t ncomplex, int nfield, uint64_t seed, uint32_t stream) {
  const size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x;
  const int f = blockIdx.y;
  if (i * 2 >= ncomplex || f >= nfield) return;
  uint4 r = philox4x32_10(make_uint4(uint32_t(i), uint32_t(i >> 32), uint32_t(f), stream), make_uint2(uint32_t(seed), uint32_t(seed >> 32)));
  const double inv = 1.0 / 4294967296.0;
  double u1 = (double(r.x) + 0.5) * inv, u2 = (double(r.y) + 0.5) * inv;
  double u3 = (double(r.z) + 0.5) * inv, u4 = (double(r.w) + 0.5) * inv;
  double rad1 = sqrt(-log(u1)), rad2 = sqrt(-log(u3));  // |z|^2 ~ Exp(1)
  double* o = out + size_t(f) * ncomplex * 2;
  o[4 * i + 0] = rad1 * cos(6.283185307179586 * u2);
  o[4 * i + 1] = rad1 * sin(6.283185307179586 * u2);
  if (2 * i + 1 < ncomplex) {
    o[4 * i + 2] = rad2 * cos(6.283185307179586 * u4);
    o[4 * i + 3] = rad2 * sin(6.283185307179586 * u4);
  }
}

void launch_gaussian(hipStream_t st, double* out, size_t ncomplex, int nfield, uint64_t seed, uint32_t stream) {
  size_t n = (ncomplex + 1) / 2;
  hipLaunchKernelGGL(k_gaussian, dim3(unsigned((n + 255) / 256), nfield), dim3(256), 0, st, out, ncomplex, nfield, seed, stream);
}

}  // namespace psms
