// Exact block determinants (the block filter of Sec. 3, eq. 4step step 1): the
// even-odd reduced operator of every Dirichlet block, A_b = 1 - kappa^2 H_eo H_oe
// restricted to the block's even sites (det D_b = det A_b because D_b has unit
// diagonal blocks in the even-odd order), assembled as dense matrices and factorised
// by a batched right-looking blocked LU in FP64 on the matrix cores.
//
// Matrices: complex, n x n with n = 6 V_b padded to npad (a multiple of 64, identity on
// the padding), stored column-major as two planes per matrix: re[npad*npad], then im.
// The LU runs without row exchanges: A_b = 1 - X with X the two-hop transport inside a
// block, whose leading minors are those of the same operator on smaller Dirichlet
// regions. Every pivot is checked: a pivot whose modulus falls below 1e-8 (or is not
// finite) is reported, and the host refuses the result.
//
// One panel step k (tiles of 64):
//   k_lu_diag   A_kk = L_kk U_kk in LDS, sum of ln u_cc, explicit inverses of L_kk, U_kk;
//   k_lu_gemm   L_ik = A_ik U_kk^-1 and U_kj = L_kk^-1 A_kj (tiles right of / below);
//   k_lu_gemm   A_ij -= L_ik U_kj (trailing tiles).
// The tile products run on v_mfma_f64_16x16x4_f64: a complex product is four real
// ones (re re - im im, re im + im re), the minus sign carried by the operand.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace psms {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int LU_T = 64;  // tile edge

// ----------------------------------------------------------------- assembly
// e[r] (FP64 internal layout, nr fields): for column k0 + r, the unit vector at the
// block's even site i = k / 12, spin-colour component k % 12, in every block at once
// (blocks do not interact under the block-restricted hops). The field is zeroed first.
__global__ void k_lu_units(Geo g, double2* __restrict__ e, int k0, int nr, int n) {
  const int blk = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (blk >= g.nblk || r >= nr) return;
  const int k = k0 + r;
  if (k >= n) return;
  const int i = k / 12, a = k % 12;
  const size_t Vh = g.Vh;
  e[size_t(r) * 24 * Vh + size_t(a) * Vh + size_t(blk) * g.Vbh + i] = make_double2(1.0, 0.0);
}

// Column k0 + r of A_b for blocks [b0, b0 + nb): rows j*12 + a' from y's even sites of
// the block (y = -kappa^2 H_eo H_oe e), plus the identity.
__global__ void k_lu_scatter(Geo g, const double2* __restrict__ y, double* __restrict__ M, int k0, int nr, int n,
                             int npad, int b0, int nb) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;  // j * 12 + a'
  const int r = blockIdx.y;
  const int bl = blockIdx.z;
  if (row >= n || r >= nr || bl >= nb) return;
  const int k = k0 + r;
  if (k >= n) return;
  const int j = row / 12, a = row % 12;
  const size_t Vh = g.Vh;
  const double2 v = y[size_t(r) * 24 * Vh + size_t(a) * Vh + size_t(b0 + bl) * g.Vbh + j];
  const size_t plane = size_t(npad) * npad;
  double* m = M + size_t(bl) * 2 * plane;
  m[size_t(k) * npad + row] = v.x + (row == k ? 1.0 : 0.0);
  m[plane + size_t(k) * npad + row] = v.y;
}

// Zero every matrix, with ones on the padded diagonal (rows and columns >= n).
__global__ void k_lu_init(double* __restrict__ M, int n, int npad, int nmat) {
  const size_t plane = size_t(npad) * npad;
  const size_t tot = 2 * plane * nmat;
  for (size_t t = size_t(blockIdx.x) * blockDim.x + threadIdx.x; t < tot; t += size_t(gridDim.x) * blockDim.x) {
    const size_t w = t % (2 * plane);
    const size_t col = (w % plane) / npad, row = (w % plane) % npad;
    M[t] = (w < plane && row == col && int(row) >= n) ? 1.0 : 0.0;
  }
}

void launch_lu_units(hipStream_t st, const Geo& g, double2* e, int k0, int nr, int n) {
  dim3 grid((g.nblk + 255) / 256, nr);
  hipLaunchKernelGGL(k_lu_units, grid, dim3(256), 0, st, g, e, k0, nr, n);
}

void launch_lu_scatter(hipStream_t st, const Geo& g, const double2* y, double* M, int k0, int nr, int n, int npad, int b0,
                       int nb) {
  dim3 grid((n + 255) / 256, nr, nb);
  hipLaunchKernelGGL(k_lu_scatter, grid, dim3(256), 0, st, g, y, M, k0, nr, n, npad, b0, nb);
}

void launch_lu_init(hipStream_t st, double* M, int n, int npad, int nmat) {
  hipLaunchKernelGGL(k_lu_init, dim3(4096), dim3(256), 0, st, M, n, npad, nmat);
}

// ----------------------------------------------------------------- diagonal tile
// One workgroup per matrix: LU of the 64 x 64 tile (k, k) in LDS without exchanges, the
// sum of ln u_cc into logdet[mat] (sum of ln|u|, sum of arg u), the smallest |u_cc| into
// minpiv[mat], and L_kk^-1 (unit lower) and U_kk^-1 into inv[mat] (two 64 x 64 complex
// tiles, column-major, planes re then im: L^-1 first, U^-1 second).
__global__ void __launch_bounds__(256) k_lu_diag(double* __restrict__ M, int npad, int k, double2* __restrict__ logdet,
                                                 double* __restrict__ minpiv, double* __restrict__ inv) {
  __shared__ double Are[LU_T][LU_T + 1], Aim[LU_T][LU_T + 1];  // [row][col]
  __shared__ double Xre[LU_T][LU_T + 1], Xim[LU_T][LU_T + 1];
  __shared__ double pre[4][LU_T], pim[4][LU_T];
  const int t = threadIdx.x;
  const int mat = blockIdx.x;
  const size_t plane = size_t(npad) * npad;
  const double* m = M + size_t(mat) * 2 * plane;
  const size_t base = size_t(k) * LU_T * npad + size_t(k) * LU_T;
  for (int e = t; e < LU_T * LU_T; e += 256) {
    const int c = e / LU_T, r = e % LU_T;
    Are[r][c] = m[base + size_t(c) * npad + r];
    Aim[r][c] = m[plane + base + size_t(c) * npad + r];
  }
  __syncthreads();
  for (int c = 0; c < LU_T; ++c) {
    const double pr = Are[c][c], pi = Aim[c][c];
    const double d = pr * pr + pi * pi;
    const double ir = pr / d, ii = -pi / d;  // 1 / u_cc
    if (t > c && t < LU_T) {
      const double a = Are[t][c], b = Aim[t][c];
      Are[t][c] = a * ir - b * ii;
      Aim[t][c] = a * ii + b * ir;
    }
    __syncthreads();
    const int w = LU_T - 1 - c;
    for (int e = t; e < w * w; e += 256) {
      const int r = c + 1 + e / w, j = c + 1 + e % w;
      const double lr = Are[r][c], li = Aim[r][c], ur = Are[c][j], ui = Aim[c][j];
      Are[r][j] -= lr * ur - li * ui;
      Aim[r][j] -= lr * ui + li * ur;
    }
    __syncthreads();
  }
  if (t == 0) {
    double sl = 0.0, sa = 0.0, mp = minpiv[mat];
    for (int c = 0; c < LU_T; ++c) {
      const double a = Are[c][c], b = Aim[c][c];
      const double ab = sqrt(a * a + b * b);
      mp = (ab < mp || ab != ab) ? ab : mp;
      sl += log(ab);
      sa += atan2(b, a);
    }
    minpiv[mat] = mp;
    const double2 o = logdet[mat];
    logdet[mat] = make_double2(o.x + sl, o.y + sa);
  }
  double* out = inv + size_t(mat) * 4 * LU_T * LU_T;
  // L^-1: X[r][c] = -sum_{m=c}^{r-1} L[r][m] X[m][c] for r > c, X[c][c] = 1 (rows ascending);
  // thread t: column c = t % 64, partial sum over m = c + q, c + q + 4, ... (q = t / 64)
  const int c = t % LU_T, q = t / LU_T;
  for (int e = t; e < LU_T * LU_T; e += 256) {
    const int rr = e / LU_T, cc = e % LU_T;
    Xre[rr][cc] = rr == cc ? 1.0 : 0.0;
    Xim[rr][cc] = 0.0;
  }
  __syncthreads();
  for (int r = 1; r < LU_T; ++r) {
    double sr = 0.0, si = 0.0;
    if (c < r)
      for (int mm = c + q; mm < r; mm += 4) {
        const double lr = Are[r][mm], li = Aim[r][mm], xr = Xre[mm][c], xi = Xim[mm][c];
        sr += lr * xr - li * xi;
        si += lr * xi + li * xr;
      }
    pre[q][c] = sr;
    pim[q][c] = si;
    __syncthreads();
    if (t < r) {
      Xre[r][t] = -(pre[0][t] + pre[1][t] + pre[2][t] + pre[3][t]);
      Xim[r][t] = -(pim[0][t] + pim[1][t] + pim[2][t] + pim[3][t]);
    }
    __syncthreads();
  }
  for (int e = t; e < LU_T * LU_T; e += 256) {
    const int cc = e / LU_T, rr = e % LU_T;
    out[size_t(cc) * LU_T + rr] = Xre[rr][cc];
    out[LU_T * LU_T + size_t(cc) * LU_T + rr] = Xim[rr][cc];
  }
  __syncthreads();
  // U^-1: X[c][c] = 1/u_cc; X[r][c] = -(sum_{m=r+1}^{c} U[r][m] X[m][c]) / u_rr for r < c
  // (rows descending)
  for (int e = t; e < LU_T * LU_T; e += 256) {
    const int rr = e / LU_T, cc = e % LU_T;
    double xr = 0.0, xi = 0.0;
    if (rr == cc) {
      const double a = Are[rr][rr], b = Aim[rr][rr], d = a * a + b * b;
      xr = a / d;
      xi = -b / d;
    }
    Xre[rr][cc] = xr;
    Xim[rr][cc] = xi;
  }
  __syncthreads();
  for (int r = LU_T - 2; r >= 0; --r) {
    double sr = 0.0, si = 0.0;
    if (c > r)
      for (int mm = r + 1 + q; mm <= c; mm += 4) {
        const double ur = Are[r][mm], ui = Aim[r][mm], xr = Xre[mm][c], xi = Xim[mm][c];
        sr += ur * xr - ui * xi;
        si += ur * xi + ui * xr;
      }
    pre[q][c] = sr;
    pim[q][c] = si;
    __syncthreads();
    if (t > r && t < LU_T) {
      const double s0 = pre[0][t] + pre[1][t] + pre[2][t] + pre[3][t];
      const double s1 = pim[0][t] + pim[1][t] + pim[2][t] + pim[3][t];
      const double a = Are[r][r], b = Aim[r][r], d = a * a + b * b;
      const double ir = a / d, ii = -b / d;
      Xre[r][t] = -(s0 * ir - s1 * ii);
      Xim[r][t] = -(s0 * ii + s1 * ir);
    }
    __syncthreads();
  }
  for (int e = t; e < LU_T * LU_T; e += 256) {
    const int cc = e / LU_T, rr = e % LU_T;
    out[2 * LU_T * LU_T + size_t(cc) * LU_T + rr] = Xre[rr][cc];
    out[3 * LU_T * LU_T + size_t(cc) * LU_T + rr] = Xim[rr][cc];
  }
}

// ----------------------------------------------------------------- tile product
// C = beta C + sgn A B for one 64 x 64 complex tile, A and B 64 x 64 (column-major
// planes: x_re[col * ld + row], x_im at + pl). Four waves, each a 32 x 32 quarter of C
// as 2 x 2 MFMA tiles of 16 x 16. Operand layout of v_mfma_f64_16x16x4_f64 (wave lane l):
// A[l % 16][l / 16], B[l / 16][l % 16]; result element v of lane l is C[4 v + l / 16][l % 16]
// (the f64 form interleaves the rows of its four result registers across the lane groups).
struct TileRef {
  const double* p;
  size_t ld, pl;
};

__device__ __forceinline__ void tile_gemm(TileRef A, TileRef B, double* C, size_t ldc, size_t plc, int beta, double sgn) {
  __shared__ double As[2][16][LU_T];  // [re/im][k][row]
  __shared__ double Bs[2][16][LU_T];  // [re/im][k][col]
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r0 = 32 * (w & 1), c0 = 32 * (w >> 1);
  d4 cre[2][2], cim[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (beta) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = r0 + 16 * i + 4 * v + (lane >> 4), col = c0 + 16 * j + (lane & 15);
          cre[i][j][v] = C[size_t(col) * ldc + row];
          cim[i][j][v] = C[plc + size_t(col) * ldc + row];
        }
      } else {
        cre[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        cim[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      }
    }
  for (int kc = 0; kc < LU_T; kc += 16) {
    // stage A[:, kc:kc+16] and B[kc:kc+16, :]
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      const int ar = e % LU_T, ak = e / LU_T;      // A: consecutive threads walk a column
      As[0][ak][ar] = sgn * A.p[size_t(kc + ak) * A.ld + ar];
      As[1][ak][ar] = sgn * A.p[A.pl + size_t(kc + ak) * A.ld + ar];
      const int bk = e % 16, bc = e / 16;          // B: consecutive threads walk 16 rows of a column
      Bs[0][bk][bc] = B.p[size_t(bc) * B.ld + kc + bk];
      Bs[1][bk][bc] = B.p[B.pl + size_t(bc) * B.ld + kc + bk];
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = As[0][kk][r0 + 16 * i + (lane & 15)];
        ai[i] = As[1][kk][r0 + 16 * i + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        br[j] = Bs[0][kk][c0 + 16 * j + (lane & 15)];
        bi[j] = Bs[1][kk][c0 + 16 * j + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cre[i][j], 0, 0, 0);
          cre[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], cre[i][j], 0, 0, 0);
          cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], cim[i][j], 0, 0, 0);
          cim[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], cim[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + 16 * i + 4 * v + (lane >> 4), col = c0 + 16 * j + (lane & 15);
        C[size_t(col) * ldc + row] = cre[i][j][v];
        C[plc + size_t(col) * ldc + row] = cim[i][j][v];
      }
}

// Panel step k, m = T - k - 1 tiles beyond the diagonal. Grid (2m, nmat): x < m gives
// L_ik = A_ik U_kk^-1 (i = k + 1 + x), x >= m gives U_kj = L_kk^-1 A_kj (j = k + 1 + x - m),
// both in place (a workgroup reads its whole tile before writing it).
__global__ void __launch_bounds__(256) k_lu_panel(double* __restrict__ M, int npad, int k, const double* __restrict__ inv) {
  const int T = npad / LU_T, m = T - k - 1;
  const int x = blockIdx.x, mat = blockIdx.y;
  const size_t plane = size_t(npad) * npad;
  double* mb = M + size_t(mat) * 2 * plane;
  const double* iv = inv + size_t(mat) * 4 * LU_T * LU_T;
  const size_t tt = size_t(LU_T) * LU_T;
  if (x < m) {
    const int i = k + 1 + x;
    double* tile = mb + size_t(k) * LU_T * npad + size_t(i) * LU_T;
    tile_gemm(TileRef{tile, size_t(npad), plane}, TileRef{iv + 2 * tt, size_t(LU_T), tt}, tile, npad, plane, 0, 1.0);
  } else {
    const int j = k + 1 + x - m;
    double* tile = mb + size_t(j) * LU_T * npad + size_t(k) * LU_T;
    tile_gemm(TileRef{iv, size_t(LU_T), tt}, TileRef{tile, size_t(npad), plane}, tile, npad, plane, 0, 1.0);
  }
}

// Trailing update of panel step k: A_ij -= L_ik U_kj for i, j > k. Grid (m * m, nmat).
__global__ void __launch_bounds__(256) k_lu_update(double* __restrict__ M, int npad, int k) {
  const int T = npad / LU_T, m = T - k - 1;
  const int i = k + 1 + blockIdx.x / m, j = k + 1 + blockIdx.x % m, mat = blockIdx.y;
  const size_t plane = size_t(npad) * npad;
  double* mb = M + size_t(mat) * 2 * plane;
  const double* L = mb + size_t(k) * LU_T * npad + size_t(i) * LU_T;
  const double* U = mb + size_t(j) * LU_T * npad + size_t(k) * LU_T;
  double* C = mb + size_t(j) * LU_T * npad + size_t(i) * LU_T;
  tile_gemm(TileRef{L, size_t(npad), plane}, TileRef{U, size_t(npad), plane}, C, npad, plane, 1, -1.0);
}

void launch_lu_factor(hipStream_t st, double* M, int npad, int nmat, double2* logdet, double* minpiv, double* inv) {
  const int T = npad / LU_T;
  for (int k = 0; k < T; ++k) {
    hipLaunchKernelGGL(k_lu_diag, dim3(nmat), dim3(256), 0, st, M, npad, k, logdet, minpiv, inv);
    const int m = T - k - 1;
    if (m == 0) break;
    hipLaunchKernelGGL(k_lu_panel, dim3(2 * m, nmat), dim3(256), 0, st, M, npad, k, (const double*)inv);
    hipLaunchKernelGGL(k_lu_update, dim3(m * m, nmat), dim3(256), 0, st, M, npad, k);
  }
}

}  // namespace psms
