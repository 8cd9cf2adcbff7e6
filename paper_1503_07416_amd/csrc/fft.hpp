// FP64 periodic convolution of Eq. discrete_convolution through the DFT:
// (J * rho) = IDFT( h^2 DFT(J) . DFT(rho) ).  A 2-D DFT of an n x n grid is
// row DFTs, a transpose, row DFTs; every row transform runs in LDS as a
// radix-2 Stockham autosort FFT (n = 2^p, p <= 12; a 4096-point complex FP64
// row and its ping-pong buffer take 128 KiB of the 160 KiB LDS).
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

// Inverse row DFT, real part times scale into a real grid.
__global__ void k_fft_rows_real_inv(const double2* __restrict__ in, double* __restrict__ out, int n,
                                    double scale) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + n;
  const size_t row = (size_t)blockIdx.x * n;
  for (int t = threadIdx.x; t < n; t += blockDim.x) a[t] = in[row + t];
  __syncthreads();
  double2* r = fft_lds(a, b, n, true);
  for (int t = threadIdx.x; t < n; t += blockDim.x) out[row + t] = r[t].x * scale;
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
