// Register-only VALU rate probes on gfx950: the ceilings the roofline of the
// NTT and multiply-accumulate kernels is priced against, measured on the
// device the library runs on. Each probe runs independent dependency chains
// of one instruction class in registers (no memory traffic inside the timed
// loop) over enough workgroups to fill every compute unit:
//   simple : 32-bit integer add/sub (v_add_u32 / v_sub_u32)
//   mul    : 32-bit integer multiplies (v_mul_lo_u32 / v_mul_hi_u32)
//   mad64  : v_mad_u64_u32, the multiply-accumulate's instruction
//   bfly   : the inverse NTT's Gentleman-Sande butterfly with a Shoup twiddle,
//            compiled from the same inv_pass template as the inverse kernels
//            (16 coefficients per thread, 4 stages per pass, per-lane twiddles
//            in registers)
#include "hc_device.h"

namespace hc {

constexpr int kProbeChains = 16;

// The simple-op probe also reads the shader clock counter at its start and
// end: thread 0 of each workgroup stores the elapsed cycles at out[1 + block]
// (all workgroups are resident at once at this register count, so the
// elapsed cycles over the launch's duration give the engine clock under load).
__global__ __launch_bounds__(256) void k_probe_simple(uint32_t *out, uint32_t iters, uint32_t a, uint32_t b) {
  const uint64_t c0 = clock64();
  uint32_t x[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) x[k] = threadIdx.x + k;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[k]) : "v"(a));
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) asm volatile("v_sub_u32 %0, %0, %1" : "+v"(x[k]) : "v"(b));
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s ^= x[k];
  if (s == 0x9e3779b9u) out[0] = s;  // keeps the chains live; practically never stores
  const uint64_t c1 = clock64();
  if (threadIdx.x == 0) out[1 + blockIdx.x] = (uint32_t)(c1 - c0);
}

__global__ __launch_bounds__(256) void k_probe_mul(uint32_t *out, uint32_t iters, uint32_t a, uint32_t b) {
  uint32_t x[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) x[k] = threadIdx.x + k + 1;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[k]) : "v"(a));
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[k]) : "v"(b));
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s ^= x[k];
  if (s == 0x9e3779b9u) out[0] = s;
}

__global__ __launch_bounds__(256) void k_probe_mad64(uint32_t *out, uint32_t iters, uint32_t a, uint32_t b) {
  uint64_t acc[kProbeChains];
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) acc[k] = threadIdx.x + k;
  const uint32_t x = a + threadIdx.x;
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
      acc[k] += (uint64_t)x * (b + k);
      asm volatile("" : "+v"(acc[k]));
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kProbeChains; ++k) s ^= acc[k];
  if (s == 0x9e3779b97f4a7c15ull) out[0] = (uint32_t)s;
}

// Twiddles for the butterfly probe: {w, floor(w 2^32 / q)} pairs, any w < q.
// Two per stage, in registers (per-lane values, as in the first inverse
// passes): the instruction sequence is that of the kernels, and the probe
// needs few enough registers for 8 waves per SIMD.
struct ProbeTw {
  uint32_t w[4][2], wp[4][2];
  __device__ __forceinline__ uint2 operator()(int bb, int u) const {
    return make_uint2(w[bb][(u >> 1) & 1], wp[bb][(u >> 1) & 1]);
  }
};

__global__ __launch_bounds__(256) void k_probe_bfly(uint32_t *out, uint32_t iters, uint32_t q, const uint2 *tw) {
  ProbeTw t;
#pragma unroll
  for (int bb = 0; bb < 4; ++bb)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const uint2 v = tw[(bb * 2 + u + threadIdx.x) & 63];
      t.w[bb][u] = v.x;
      t.wp[bb][u] = v.y;
    }
  uint32_t v[1][16];
#pragma unroll
  for (int u = 0; u < 16; ++u) v[0][u] = (threadIdx.x * 16 + u) % q;
  for (uint32_t it = 0; it < iters; ++it) {
    // stages on index bits 0..3 of a 2^13-point transform (none is the last
    // stage, so every butterfly takes the general form): 32 butterflies
    inv_pass<13, 4, 0, 4, 0, 1>(v, t, q, 0u, 0u, 0u, 0u);
  }
  uint32_t s = 0;
#pragma unroll
  for (int u = 0; u < 16; ++u) s ^= v[0][u];
  if (s == 0x9e3779b9u) out[0] = s;
}

hipError_t launch_probe(int kind, uint32_t nwg, uint32_t iters, uint32_t q, const uint2 *tw, uint32_t *out,
                        hipStream_t st) {
  switch (kind) {
    case 0:
      hipLaunchKernelGGL(k_probe_simple, dim3(nwg), dim3(256), 0, st, out, iters, 3u, 5u);
      break;
    case 1:
      hipLaunchKernelGGL(k_probe_mul, dim3(nwg), dim3(256), 0, st, out, iters, 0x9e3779b1u, 0x85ebca77u);
      break;
    case 2:
      hipLaunchKernelGGL(k_probe_mad64, dim3(nwg), dim3(256), 0, st, out, iters, 0x9e3779b1u, 0x85ebca77u);
      break;
    case 3:
      hipLaunchKernelGGL(k_probe_bfly, dim3(nwg), dim3(256), 0, st, out, iters, q, tw);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace hc

// ---------------------------------------------------------------- host entry point
#include <algorithm>
#include <vector>

#include "hc_objects.h"

namespace {
// One timed launch of probe `kind` (after one untimed warm-up launch) in ms.
hipError_t time_probe(int kind, uint32_t nwg, uint32_t iters, uint32_t q, const uint2 *tw, uint32_t *out,
                      hipStream_t st, float *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hc::launch_probe(kind, nwg, iters, q, tw, out, st);
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = hc::launch_probe(kind, nwg, iters, q, tw, out, st);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}
}  // namespace

extern "C" hc_status hc_valu_probe(int hip_device, hc_valu_rates *out) {
  if (!out) return hc::fail(HC_EINVAL, "hc_valu_probe: null output");
  hc::DeviceGuard dg(hip_device);
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, hip_device);
  if (e != hipSuccess) return hc::hip_fail(e, "hc_valu_probe: device properties");
  const uint32_t cus = (uint32_t)prop.multiProcessorCount;
  const uint32_t nwg = cus * 8;  // 8 four-wave workgroups per compute unit
  // a prime below 2^30 and Shoup twiddle pairs for it (any residues will do)
  const uint32_t q = 1073692673u;
  std::vector<uint2> htw(64);
  for (uint32_t k = 0; k < 64; ++k) {
    const uint32_t w = (uint32_t)((0x9e3779b97f4a7c15ull * (k + 1)) % q);
    htw[k] = make_uint2(w, (uint32_t)(((uint64_t)w << 32) / q));
  }
  uint2 *dtw = nullptr;
  uint32_t *dout = nullptr;
  hipStream_t st = nullptr;
  e = hipMalloc((void **)&dtw, 64 * sizeof(uint2));
  if (e == hipSuccess) e = hipMalloc((void **)&dout, (size_t)(1 + nwg) * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpy(dtw, htw.data(), 64 * sizeof(uint2), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreate(&st);
  // lane operations per thread per loop turn: 2 x 16 chains (simple, mul),
  // 16 chains (mad64); butterflies: 32 per turn
  const uint32_t iters[4] = {4096, 2048, 2048, 512};
  const double per_turn[4] = {32.0, 32.0, 16.0, 32.0};
  double rate[4] = {0, 0, 0, 0};
  double clock_meas = 0.0;
  for (int k = 0; k < 4 && e == hipSuccess; ++k) {
    float ms = 0.f;
    e = time_probe(k, nwg, iters[k], q, dtw, dout, st, &ms);
    if (e == hipSuccess) rate[k] = (double)nwg * 256.0 * iters[k] * per_turn[k] / (ms * 1e-3);
    if (e == hipSuccess && k == 0) {
      std::vector<uint32_t> cyc(nwg);
      e = hipMemcpy(cyc.data(), dout + 1, nwg * sizeof(uint32_t), hipMemcpyDeviceToHost);
      double mx = 0;
      for (uint32_t c : cyc) mx = std::max(mx, (double)c);
      if (e == hipSuccess && ms > 0) clock_meas = mx / (ms * 1e-3);
    }
  }
  if (st) (void)hipStreamDestroy(st);
  if (dtw) (void)hipFree(dtw);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return hc::hip_fail(e, "hc_valu_probe");
  out->simple_ops_per_s = rate[0];
  out->mul_ops_per_s = rate[1];
  out->mad64_ops_per_s = rate[2];
  out->butterflies_per_s = rate[3];
  out->compute_units = cus;
  out->clock_hz = (double)prop.clockRate * 1e3;
  out->measured_clock_hz = clock_meas;
  return HC_OK;
}
