// State initialisation and FP64 export kernels (not on the per-step path).
//
// Initial populations are the equilibrium of the initial fields (Sec. 3,
// eq. f-eq): f^0 = wdot - A0 w, f^k = Ak w with A0 = 2 lambda / c^2 and
// Ak = lambda / (2 c^2).  Shifted storage keeps g = f - E(w_stored) with the
// static equilibrium E^0 = -A0 w, E^k = Ak w of the stored (FP32) w.
#include "lbm_internal.hpp"

namespace lbmk {
namespace {

template <typename S> __device__ __forceinline__ S cvt_out(double x) { return static_cast<S>(x); }
template <> __device__ __forceinline__ _Float16 cvt_out<_Float16>(double x) {
  return static_cast<_Float16>(static_cast<float>(x));
}
template <> __device__ __forceinline__ __bf16 cvt_out<__bf16>(double x) {
  return static_cast<__bf16>(static_cast<float>(x));
}
__device__ __forceinline__ double cvt_in(double x) { return x; }
__device__ __forceinline__ double cvt_in(float x) { return x; }
__device__ __forceinline__ double cvt_in(_Float16 x) { return static_cast<float>(x); }
__device__ __forceinline__ double cvt_in(__bf16 x) { return static_cast<float>(x); }

template <typename S, typename W, bool SHIFT>
__global__ void init_rows_kernel(S *f, W *w, W *w2, Plate p, int row0, int nrows, const double *w0,
                                 const double *wd0, double A0, double Ak) {
#pragma clang fp contract(off)
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nrows * p.pitch;
  if (t >= n) return;
  const int jj = (int)(t / p.pitch);
  const int i = (int)(t % p.pitch);
  const size_t x = (size_t)(row0 + jj) * p.pitch + i;
  double wv = 0.0, wdv = 0.0;
  if (i < p.nx) {
    if (w0) wv = w0[(size_t)jj * p.nx + i];
    if (wd0) wdv = wd0[(size_t)jj * p.nx + i];
  }
  if (!SHIFT) {
    f[x] = cvt_out<S>(wdv - A0 * wv);
    for (int a = 1; a < 5; ++a) f[a * p.plane + x] = cvt_out<S>(Ak * wv);
    w[x] = static_cast<W>(wv);
    w2[x] = static_cast<W>(wv);
  } else {
    const W ws = static_cast<W>(wv);
    const double dw = wv - (double)ws;  // part of w0 that the stored w cannot hold
    f[x] = cvt_out<S>(wdv - A0 * dw);
    for (int a = 1; a < 5; ++a) f[a * p.plane + x] = cvt_out<S>(Ak * dw);
    w[x] = ws;
    w2[x] = ws;
  }
}

template <typename S, typename W, bool SHIFT>
__global__ void export_rows_kernel(const S *f, const W *w, Plate p, int row0, int nrows, double A0,
                                   double Ak, double *w_out, double *wd_out, double *f_out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)nrows * p.nx;
  if (t >= n) return;
  const int jj = (int)(t / p.nx);
  const int i = (int)(t % p.nx);
  const size_t x = (size_t)(row0 + jj) * p.pitch + i;
  const double wv = cvt_in(w[x]);
  if (w_out) w_out[t] = wv;
  double v[5];
  for (int a = 0; a < 5; ++a) v[a] = cvt_in(f[a * p.plane + x]);
  if (wd_out) {
    double acc = 0.0;
    for (int a = 0; a < 5; ++a) acc += v[a];
    wd_out[t] = acc;
  }
  if (f_out) {
    for (int a = 0; a < 5; ++a) {
      double fa = v[a];
      if (SHIFT) fa += (a == 0) ? -A0 * wv : Ak * wv;
      f_out[(size_t)a * n + t] = fa;
    }
  }
}

__global__ void export_mask_kernel(const uint32_t *mV, const uint32_t *mH, Plate p, uint8_t *v_out,
                                   uint8_t *h_out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)p.nx * p.ny) return;
  const int j = (int)(t / p.nx), i = (int)(t % p.nx);
  const size_t wofs = (size_t)j * p.mw + (i >> 5);
  if (v_out) v_out[t] = (mV[wofs] >> (i & 31)) & 1u;
  if (h_out) h_out[t] = (mH[wofs] >> (i & 31)) & 1u;
}

__global__ void zero_kernel(uint4 *p, size_t n16, uint8_t *tail, size_t ntail) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t k = t; k < n16; k += stride) p[k] = make_uint4(0, 0, 0, 0);
  if (t < ntail) tail[t] = 0;
}

unsigned blocks_for(size_t n) { return (unsigned)((n + 255) / 256); }

template <typename S, typename W, bool SHIFT>
hipError_t init_t(void *f, void *w, void *w2, const Plate &p, int row0, int nrows, const double *w0,
                  const double *wd0, double A0, double Ak, hipStream_t st) {
  const size_t n = (size_t)nrows * p.pitch;
  hipLaunchKernelGGL((init_rows_kernel<S, W, SHIFT>), dim3(blocks_for(n)), dim3(256), 0, st,
                     static_cast<S *>(f), static_cast<W *>(w), static_cast<W *>(w2), p, row0, nrows,
                     w0, wd0, A0, Ak);
  return hipGetLastError();
}

template <typename S, typename W, bool SHIFT>
hipError_t export_t(const void *f, const void *w, const Plate &p, int row0, int nrows, double A0,
                    double Ak, double *w_out, double *wd_out, double *f_out, hipStream_t st) {
  const size_t n = (size_t)nrows * p.nx;
  hipLaunchKernelGGL((export_rows_kernel<S, W, SHIFT>), dim3(blocks_for(n)), dim3(256), 0, st,
                     static_cast<const S *>(f), static_cast<const W *>(w), p, row0, nrows, A0, Ak,
                     w_out, wd_out, f_out);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_init_rows(Store s, void *f, void *w, void *w2, const Plate &p, int row0,
                            int nrows, const double *w0, const double *wd0, double A0, double Ak,
                            hipStream_t st) {
  switch (s) {
    case Store::F64: return init_t<double, double, false>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
    case Store::F64S: return init_t<double, double, true>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
    case Store::F32_PLAIN: return init_t<float, float, false>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
    case Store::F32S: return init_t<float, float, true>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
    case Store::F16S: return init_t<_Float16, float, true>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
    case Store::BF16S: return init_t<__bf16, float, true>(f, w, w2, p, row0, nrows, w0, wd0, A0, Ak, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_export_rows(Store s, const void *f, const void *w, const Plate &p, int row0,
                              int nrows, double A0, double Ak, double *w_out, double *wd_out,
                              double *f_out, hipStream_t st) {
  switch (s) {
    case Store::F64: return export_t<double, double, false>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
    case Store::F64S: return export_t<double, double, true>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
    case Store::F32_PLAIN: return export_t<float, float, false>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
    case Store::F32S: return export_t<float, float, true>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
    case Store::F16S: return export_t<_Float16, float, true>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
    case Store::BF16S: return export_t<__bf16, float, true>(f, w, p, row0, nrows, A0, Ak, w_out, wd_out, f_out, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_export_mask(const uint32_t *mV, const uint32_t *mH, const Plate &p, uint8_t *v_out,
                              uint8_t *h_out, hipStream_t st) {
  const size_t n = (size_t)p.nx * p.ny;
  hipLaunchKernelGGL(export_mask_kernel, dim3(blocks_for(n)), dim3(256), 0, st, mV, mH, p, v_out, h_out);
  return hipGetLastError();
}

hipError_t launch_zero(void *ptr, size_t bytes, hipStream_t st) {
  const size_t n16 = bytes / 16, ntail = bytes % 16;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) blocks = 1;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, static_cast<uint4 *>(ptr),
                     n16, static_cast<uint8_t *>(ptr) + n16 * 16, ntail);
  return hipGetLastError();
}

}  // namespace lbmk
