// Metadynamics bias of Eq. 1 on the path variables (s, z), kept on a
// regular grid as in the paper's runs, and its gradient on the atoms.
//
// Every node of the (s, z) grid holds the exact sum of the deposited hills
// w exp(-(s - s_k)^2 / (2 sigma_s^2) - (z - z_k)^2 / (2 sigma_z^2)) and its
// derivatives dV/ds, dV/dz, d2V/dsdz (FP64, SoA planes [4][ns][nz]).  A
// deposit reads the CV values from device memory (no host round trip) and
// updates every node, one thread per node, so deposits are ordered by the
// stream.  Between nodes the bias is the bicubic Hermite interpolant of the
// four corner values; outside the grid it is zero.  The atom gradient is
// dV/dx = dV/ds ds/dx + dV/dz dz/dx, one workgroup per 256 outputs (each
// workgroup interpolates the same cell itself).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "pcv.h"
#include "pcv_host_util.h"
#include "pcv_internal.h"

namespace pcv {

namespace {

struct BiasGrid {
  double s_min, s_max, z_min, z_max, hs, hz, height, sigma_s, sigma_z;
  int ns, nz;
  double* data;   // [4][ns][nz]
};

__global__ __launch_bounds__(256) void bias_deposit_kernel(BiasGrid g, const double* __restrict__ sz) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int nodes = g.ns * g.nz;
  if (idx >= nodes) return;
  const double s0 = ldg(sz), z0 = ldg(sz + 1);
  if (!isfinite(s0) || !isfinite(z0)) return;
  const int i = idx / g.nz, j = idx - i * g.nz;
  const double s = g.s_min + i * g.hs, z = g.z_min + j * g.hz;
  const double ds = s - s0, dz = z - z0;
  const double v = g.height * exp(-ds * ds / (2.0 * g.sigma_s * g.sigma_s) - dz * dz / (2.0 * g.sigma_z * g.sigma_z));
  const double a = -ds / (g.sigma_s * g.sigma_s), b = -dz / (g.sigma_z * g.sigma_z);
  double* d = g.data;
  d[idx] += v;
  d[(size_t)nodes + idx] += a * v;
  d[2 * (size_t)nodes + idx] += b * v;
  d[3 * (size_t)nodes + idx] += a * b * v;
}

// Cubic Hermite basis on [0, 1]: value weights of the left / right node
// (h[0], h[2]) and slope weights (h[1], h[3]); dh: their derivatives.
__device__ __forceinline__ void hermite4(double t, double h[4], double dh[4]) {
  const double t2 = t * t, t3 = t2 * t;
  h[0] = 2 * t3 - 3 * t2 + 1;
  h[1] = t3 - 2 * t2 + t;
  h[2] = -2 * t3 + 3 * t2;
  h[3] = t3 - t2;
  dh[0] = 6 * t2 - 6 * t;
  dh[1] = 3 * t2 - 4 * t + 1;
  dh[2] = -6 * t2 + 6 * t;
  dh[3] = 3 * t2 - 2 * t;
}

// (V, dV/ds, dV/dz) and the in-range flag at (s, z).
__device__ void bias_interpolate(const BiasGrid& g, double s, double z, double out[3], int& ok) {
  out[0] = out[1] = out[2] = 0.0;
  ok = (s >= g.s_min && s <= g.s_max && z >= g.z_min && z <= g.z_max) ? 1 : 0;
  if (!ok) return;
  const int i = min((int)floor((s - g.s_min) / g.hs), g.ns - 2);
  const int j = min((int)floor((z - g.z_min) / g.hz), g.nz - 2);
  const double t = (s - (g.s_min + i * g.hs)) / g.hs;
  const double u = (z - (g.z_min + j * g.hz)) / g.hz;
  double ht[4], dt[4], hu[4], du[4];
  hermite4(t, ht, dt);
  hermite4(u, hu, du);
  const size_t nodes = (size_t)g.ns * g.nz;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const size_t at = (size_t)(i + a) * g.nz + (j + b);
      const double f = g.data[at], fs = g.data[nodes + at], fz = g.data[2 * nodes + at],
                   fsz = g.data[3 * nodes + at];
      const double coef[2][2] = {{f, g.hz * fz}, {g.hs * fs, g.hs * g.hz * fsz}};
      for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
          const double Ht = ht[2 * a + p], Dt = dt[2 * a + p], Hu = hu[2 * b + q], Du = du[2 * b + q];
          out[0] += coef[p][q] * Ht * Hu;
          out[1] += coef[p][q] * Dt / g.hs * Hu;
          out[2] += coef[p][q] * Ht * Du / g.hz;
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void bias_gradient_kernel(BiasGrid g, const double* __restrict__ sz, int m,
                                                            const T* __restrict__ ds, const T* __restrict__ dz,
                                                            T* __restrict__ out, double* __restrict__ v,
                                                            int* __restrict__ in_range) {
  __shared__ double sv[3];
  if (threadIdx.x == 0) {
    double r[3];
    int ok;
    bias_interpolate(g, ldg(sz), ldg(sz + 1), r, ok);
    sv[0] = r[0];
    sv[1] = r[1];
    sv[2] = r[2];
    if (blockIdx.x == 0) {
      if (v) {
        v[0] = r[0];
        v[1] = r[1];
        v[2] = r[2];
      }
      if (in_range) *in_range = ok;
    }
  }
  __syncthreads();
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < m && out) out[k] = (T)(sv[1] * (double)ds[k] + sv[2] * (double)dz[k]);
}

}  // namespace

}  // namespace pcv

using namespace pcv;

struct pcv_bias {
  pcv_bias_options opt{};
  hipStream_t stream = nullptr;
  BiasGrid g{};
  DevMem mem;
  long long hills = 0;
  std::string err;
};

static pcv_status bias_fail(pcv_bias* b, pcv_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

extern "C" pcv_status pcv_bias_create(pcv_bias** out, const pcv_bias_options* o) {
  if (!out || !o) return PCV_EINVAL;
  *out = nullptr;
  if (o->ns < 2 || o->nz < 2 || !(o->s_max > o->s_min) || !(o->z_max > o->z_min) || !std::isfinite(o->s_min) ||
      !std::isfinite(o->s_max) || !std::isfinite(o->z_min) || !std::isfinite(o->z_max) || !(o->sigma_s > 0.0) ||
      !(o->sigma_z > 0.0) || !std::isfinite(o->height) || !std::isfinite(o->sigma_s) || !std::isfinite(o->sigma_z))
    return PCV_EINVAL;
  if ((long long)o->ns * o->nz > (1LL << 28)) return PCV_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || o->device < 0 || o->device >= ndev) return PCV_EHIP;
  if (hipSetDevice(o->device) != hipSuccess) return PCV_EHIP;
  pcv_bias* b = new pcv_bias();
  b->opt = *o;
  b->stream = (hipStream_t)o->stream;
  BiasGrid& g = b->g;
  g.s_min = o->s_min;
  g.s_max = o->s_max;
  g.z_min = o->z_min;
  g.z_max = o->z_max;
  g.ns = o->ns;
  g.nz = o->nz;
  g.hs = (o->s_max - o->s_min) / (o->ns - 1);
  g.hz = (o->z_max - o->z_min) / (o->nz - 1);
  g.height = o->height;
  g.sigma_s = o->sigma_s;
  g.sigma_z = o->sigma_z;
  const size_t bytes = (size_t)4 * g.ns * g.nz * sizeof(double);
  hipError_t e = b->mem.alloc((void**)&g.data, bytes);
  if (e == hipSuccess) e = hipMemset(g.data, 0, bytes);
  if (e != hipSuccess) {
    delete b;
    return e == hipErrorOutOfMemory ? PCV_ENOMEM : PCV_EHIP;
  }
  *out = b;
  return PCV_OK;
}

extern "C" pcv_status pcv_bias_destroy(pcv_bias* b) {
  if (!b) return PCV_OK;
  (void)hipSetDevice(b->opt.device);
  (void)hipStreamSynchronize(b->stream);
  b->mem.release();
  delete b;
  return PCV_OK;
}

extern "C" pcv_status pcv_bias_deposit(pcv_bias* b, const double* sz_dev) {
  if (!b) return PCV_EINVAL;
  if (!sz_dev) return bias_fail(b, PCV_EINVAL, "sz_dev is required");
  const int nodes = b->g.ns * b->g.nz;
  hipLaunchKernelGGL(bias_deposit_kernel, dim3((nodes + 255) / 256), dim3(256), 0, b->stream, b->g, sz_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bias_fail(b, PCV_EHIP, std::string("bias deposit: ") + hipGetErrorString(e));
  b->hills += 1;
  return PCV_OK;
}

extern "C" pcv_status pcv_bias_gradient(pcv_bias* b, const double* sz_dev, int n_atoms, int precision,
                                        const void* ds_dx, const void* dz_dx, void* grad_out, double* v_dev,
                                        int* in_range_dev) {
  if (!b) return PCV_EINVAL;
  if (!sz_dev || n_atoms < 0 || (precision != PCV_FP32 && precision != PCV_FP64))
    return bias_fail(b, PCV_EINVAL, "bad arguments");
  if (grad_out && n_atoms > 0 && (!ds_dx || !dz_dx))
    return bias_fail(b, PCV_EINVAL, "ds_dx and dz_dx are required for grad_out");
  if (n_atoms > (1 << 28) / 3) return bias_fail(b, PCV_ESHAPE, "n_atoms too large");
  const int m = grad_out ? 3 * n_atoms : 0;
  const int blocks = std::max(1, (m + 255) / 256);
  if (precision == PCV_FP32)
    hipLaunchKernelGGL(bias_gradient_kernel<float>, dim3(blocks), dim3(256), 0, b->stream, b->g, sz_dev, m,
                       (const float*)ds_dx, (const float*)dz_dx, (float*)grad_out, v_dev, in_range_dev);
  else
    hipLaunchKernelGGL(bias_gradient_kernel<double>, dim3(blocks), dim3(256), 0, b->stream, b->g, sz_dev, m,
                       (const double*)ds_dx, (const double*)dz_dx, (double*)grad_out, v_dev, in_range_dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return bias_fail(b, PCV_EHIP, std::string("bias gradient: ") + hipGetErrorString(e));
  return PCV_OK;
}

extern "C" pcv_status pcv_bias_hills(const pcv_bias* b, long long* count) {
  if (!b || !count) return PCV_EINVAL;
  *count = b->hills;
  return PCV_OK;
}

extern "C" pcv_status pcv_bias_get_grid(pcv_bias* b, double* host_out) {
  if (!b || !host_out) return PCV_EINVAL;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return bias_fail(b, PCV_EHIP, "stream synchronise failed");
  const size_t bytes = (size_t)4 * b->g.ns * b->g.nz * sizeof(double);
  if (hipMemcpy(host_out, b->g.data, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return bias_fail(b, PCV_EHIP, "grid copy failed");
  return PCV_OK;
}

extern "C" const char* pcv_bias_last_error(const pcv_bias* b) { return b ? b->err.c_str() : "null bias"; }
