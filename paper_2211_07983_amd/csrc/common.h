// Internal helpers shared by the gfx950 kernels of the MPS engine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double2 zd;  // complex double, (x, y) = (re, im)

__host__ __device__ inline zd zmk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline zd zadd(zd a, zd b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zd zsub(zd a, zd b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zd zmul(zd a, zd b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__host__ __device__ inline zd zconj(zd a) { return make_double2(a.x, -a.y); }
__host__ __device__ inline zd zscale(zd a, double s) { return make_double2(a.x * s, a.y * s); }
// acc += a * b
__host__ __device__ inline zd zfma(zd a, zd b, zd acc) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return acc;
}
// acc += conj(a) * b
__host__ __device__ inline zd zfmac(zd a, zd b, zd acc) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
  return acc;
}
__host__ __device__ inline double zabs2(zd a) { return fma(a.x, a.x, a.y * a.y); }

// Device-side bond bookkeeping of one MPS: dims[k] = bond dimension left of site
// k (dims[0] = dims[N] = 1); site k is a [dims[k]][2][dims[k+1]] tensor stored
// with capacity strides: element (l, i, r) at l*2*dcap + i*dcap + r.
struct MpsView {
  zd* B;          // [N][dcap][2][dcap]
  int* dims;      // [N+1]
  double* lam;    // [N+1][dcap]; lam[k] = Schmidt values left of site k
  int N;
  int dcap;
  __device__ __host__ inline zd* site(int n) const { return B + (size_t)n * dcap * 2 * dcap; }
  __device__ __host__ inline size_t site_elems() const { return (size_t)dcap * 2 * dcap; }
};

// ---------------------------------------------------------------------------
// A 32x32 output tile of C = A * B (complex double), 256 threads, each thread
// owning rows 2*ty+{0,1} and columns 2*tx+{0,1} of the tile.  The operands are
// fetched through functors so that one routine serves every layout; fa(i,k)
// and fb(k,j) are only called in range.  fc(i, j, acc[2][2]) receives the
// whole 2x2 register block of the thread together with its top-left index.
// ---------------------------------------------------------------------------
#define ZT_M 32
#define ZT_N 32
#define ZT_K 16

// sA/sB: LDS staging tiles of [ZT_K][ZT_M + 1] and [ZT_K][ZT_N + 1] elements.
template <typename FA, typename FB>
__device__ inline void ztile_acc_in(int M, int N, int K, int i0, int j0, FA fa, FB fb, zd acc[2][2], zd* sA, zd* sB) {
  const int t = threadIdx.x;
  const int tx = t & 15, ty = t >> 4;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = zmk(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += ZT_K) {
    for (int e = t; e < ZT_M * ZT_K; e += 256) {
      const int r = e / ZT_K, kk = e % ZT_K;
      const int gi = i0 + r, gk = k0 + kk;
      sA[kk * (ZT_M + 1) + r] = (gi < M && gk < K) ? fa(gi, gk) : zmk(0.0, 0.0);
    }
    for (int e = t; e < ZT_N * ZT_K; e += 256) {
      const int kk = e / ZT_N, cc = e % ZT_N;
      const int gk = k0 + kk, gj = j0 + cc;
      sB[kk * (ZT_N + 1) + cc] = (gk < K && gj < N) ? fb(gk, gj) : zmk(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < ZT_K; ++kk) {
      const zd a0 = sA[kk * (ZT_M + 1) + 2 * ty], a1 = sA[kk * (ZT_M + 1) + 2 * ty + 1];
      const zd b0 = sB[kk * (ZT_N + 1) + 2 * tx], b1 = sB[kk * (ZT_N + 1) + 2 * tx + 1];
      acc[0][0] = zfma(a0, b0, acc[0][0]);
      acc[0][1] = zfma(a0, b1, acc[0][1]);
      acc[1][0] = zfma(a1, b0, acc[1][0]);
      acc[1][1] = zfma(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
}

// The same with the kernel's own static LDS tiles.
template <typename FA, typename FB>
__device__ inline void ztile_acc(int M, int N, int K, int i0, int j0, FA fa, FB fb, zd acc[2][2]) {
  __shared__ zd As[ZT_K * (ZT_M + 1)];
  __shared__ zd Bs[ZT_K * (ZT_N + 1)];
  ztile_acc_in(M, N, K, i0, j0, fa, fb, acc, As, Bs);
}

#define ZT_LDS_ELEMS (ZT_K * (ZT_M + 1) + ZT_K * (ZT_N + 1))

__device__ inline int tile_row0() { return 2 * (threadIdx.x >> 4); }
__device__ inline int tile_col0() { return 2 * (threadIdx.x & 15); }

// Deterministic block reduction of one double over 256 threads.
__device__ inline double block_sum256(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}
