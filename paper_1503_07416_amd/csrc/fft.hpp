// FP64 periodic convolution of Eq. discrete_convolution through the DFT:
// (J * rho) = IDFT( h^2 DFT(J) . DFT(rho) ).  A 2-D DFT of an n x n grid is
// row DFTs, a transpose, row DFTs; every row transform runs in LDS as a
// radix-2 Stockham autosort FFT (n = 2^p, p <= 12; a 4096-point complex FP64
// row and its ping-pong buffer take 128 KiB of the 160 KiB LDS).
//
// rho and the result are real, so the convolution keeps only the x
// frequencies 0..n/2 of each row (the others are their complex conjugates):
// two real rows are transformed as one complex row x_a + i x_b, whose
// spectrum Z gives X_a(k) = (Z(k) + conj Z(n-k)) / 2 and
// X_b(k) = (Z(k) - conj Z(n-k)) / (2i); the columns of the n/2 + 1 kept
// frequencies are transformed, multiplied and transformed back; and two real
// output rows come out of one inverse complex transform of
// X_a(k) + i X_b(k), rebuilt over all k from the kept half.  Half the row
// transforms and half the column transforms of a complex convolution.
#pragma once
#include <hip/hip_runtime.h>

namespace hfz {

// Radix-2 Stockham FFT of the n points in a (ping-pong with b), natural order
// in and out.  Stage with span Ns: butterfly j pairs x[j], x[j + n/2], twiddle
// exp(-+ i pi (j mod Ns) / Ns), writes y[(j / Ns) 2 Ns + j mod Ns] and that
// + Ns.  Returns the buffer holding the result.
__device__ inline double2* fft_lds(double2* a, double2* b, int n, bool inverse) {
  const int half = n >> 1;
  const double sgn = inverse ? 1.0 : -1.0;
  for (int Ns = 1; Ns < n; Ns <<= 1) {
    for (int j = threadIdx.x; j < half; j += blockDim.x) {
      const int k = j & (Ns - 1);
      const double2 x0 = a[j];
      const double2 x1 = a[j + half];
      double sn, cs;
      sincospi(sgn * (double)k / (double)Ns, &sn, &cs);
      const double2 t = make_double2(x1.x * cs - x1.y * sn, x1.x * sn + x1.y * cs);
      const int d = ((j - k) << 1) + k;
      b[d] = make_double2(x0.x + t.x, x0.y + t.y);
      b[d + Ns] = make_double2(x0.x - t.x, x0.y - t.y);
    }
    __syncthreads();
    double2* tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

// Forward row DFT of a real grid: out[r][:] = DFT(in[r][:]).
__global__ void k_fft_rows_real_fwd(const double* __restrict__ in, double2* __restrict__ out, int n) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const size_t row = (size_t)blockIdx.x * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) a[t] = make_double2(in[row + t], 0.0);
  __syncthreads();
  double2* r = fft_lds(a, b, n, false);
  for (int t = threadIdx.x; t < n; t += blockDim.x) out[row + t] = r[t];
}

// In place on each row: forward DFT, multiply by the real multiplier row,
// inverse DFT (unnormalised).
__global__ void k_fft_rows_conv(double2* __restrict__ io, const double* __restrict__ mult, int n) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const size_t row = (size_t)blockIdx.x * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) a[t] = io[row + t];
  __syncthreads();
  double2* r = fft_lds(a, b, n, false);
  double2* o = (r == a) ? b : a;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const double m = mult[row + t];
    o[t] = make_double2(r[t].x * m, r[t].y * m);
  }
  __syncthreads();
  double2* r2 = fft_lds(o, r, n, true);
  for (int t = threadIdx.x; t < n; t += blockDim.x) io[row + t] = r2[t];
}

// Forward row DFT in place (complex rows).
__global__ void k_fft_rows_fwd(double2* __restrict__ io, int n) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const size_t row = (size_t)blockIdx.x * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) a[t] = io[row + t];
  __syncthreads();
  double2* r = fft_lds(a, b, n, false);
  for (int t = threadIdx.x; t < n; t += blockDim.x) io[row + t] = r[t];
}

// Forward DFT of two real rows per workgroup (rows 2 blockIdx.x and
// 2 blockIdx.x + 1 of the n x n grid in): frequencies 0..n/2 of each into the
// rows of out (row stride n/2 + 1).
__global__ void k_fft_rows_r2c(const double* __restrict__ in, double2* __restrict__ out, int n) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const int hx = n / 2 + 1;
  const size_t ra = (size_t)(2 * blockIdx.x) * n, rb = ra + n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) a[t] = make_double2(in[ra + t], in[rb + t]);
  __syncthreads();
  const double2* z = fft_lds(a, b, n, false);
  const size_t oa = (size_t)(2 * blockIdx.x) * hx, ob = oa + hx;
  for (int k = threadIdx.x; k < hx; k += blockDim.x) {
    const double2 zk = z[k], zn = z[(n - k) & (n - 1)];
    // X_a = (zk + conj zn) / 2, X_b = (zk - conj zn) / (2i)
    out[oa + k] = make_double2(0.5 * (zk.x + zn.x), 0.5 * (zk.y - zn.y));
    out[ob + k] = make_double2(0.5 * (zk.y + zn.y), -0.5 * (zk.x - zn.x));
  }
}

// Inverse DFT to two real rows per workgroup: in holds frequencies 0..n/2 of
// rows 2 blockIdx.x and 2 blockIdx.x + 1 (row stride n/2 + 1); the complex
// row X_a + i X_b over all k (X(n - k) = conj X(k)) is transformed back, its
// real and imaginary parts times scale are the two rows of out.
__global__ void k_fft_rows_c2r(const double2* __restrict__ in, double* __restrict__ out, int n, double scale) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const int hx = n / 2 + 1;
  const size_t ia = (size_t)(2 * blockIdx.x) * hx, ib = ia + hx;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    double2 xa, xb;
    if (k < hx) {
      xa = in[ia + k];
      xb = in[ib + k];
    } else {
      const double2 ca = in[ia + n - k], cb = in[ib + n - k];
      xa = make_double2(ca.x, -ca.y);
      xb = make_double2(cb.x, -cb.y);
    }
    a[k] = make_double2(xa.x - xb.y, xa.y + xb.x);  // X_a + i X_b
  }
  __syncthreads();
  const double2* r = fft_lds(a, b, n, true);
  const size_t ra = (size_t)(2 * blockIdx.x) * n, rb = ra + n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    out[ra + t] = r[t].x * scale;
    out[rb + t] = r[t].y * scale;
  }
}

// out = in^T for a rows x cols complex grid (row strides cols and rows),
// 32 x 32 tiles through LDS.
__global__ void k_transpose_rect(const double2* __restrict__ in, double2* __restrict__ out, int rows, int cols) {
  __shared__ double2 tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // column, row of the tile in `in`
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int x = bx + threadIdx.x, y = by + k;
    if (x < cols && y < rows) tile[k][threadIdx.x] = in[(size_t)y * cols + x];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int x = by + threadIdx.x, y = bx + k;
    if (x < rows && y < cols) out[(size_t)y * rows + x] = tile[threadIdx.x][k];
  }
}

// out = in^T for an n x n complex grid, 32 x 32 tiles through LDS.
__global__ void k_transpose(const double2* __restrict__ in, double2* __restrict__ out, int n) {
  __shared__ double2 tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int x = bx + threadIdx.x, y = by + k;
    if (x < n && y < n) tile[k][threadIdx.x] = in[(size_t)y * n + x];
  }
  __syncthreads();
  for (int k = threadIdx.y; k < 32; k += blockDim.y) {
    const int x = by + threadIdx.x, y = bx + k;
    if (x < n && y < n) out[(size_t)y * n + x] = tile[threadIdx.x][k];
  }
}

// mult = scale * Re(spec) (the DFT of the even kernel is real).
__global__ void k_real_part(const double2* __restrict__ spec, double* __restrict__ mult, size_t count,
                            double scale) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) mult[t] = spec[t].x * scale;
}

}  // namespace hfz
