// ms_peak.hip — measurement helper: the FP32 vector issue rate this library's arithmetic can
// reach on the device.  The step kernels compute with separate multiplies and adds (no fused or
// packed forms, for bit parity with the float32 oracle); this kernel runs the same instruction
// kinds on independent chains, so its rate is the ceiling of that instruction mix.

namespace {

constexpr int PEAK_CHAINS = 8;

__global__ void __launch_bounds__(64) ms_peak_fp32_kernel(float* out, int iters, float a, float b) {
    float x[PEAK_CHAINS];
#pragma unroll
    for (int k = 0; k < PEAK_CHAINS; ++k) x[k] = float(threadIdx.x) * 1e-3f + float(k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PEAK_CHAINS; ++k) x[k] = x[k] * a + b;   // one multiply, one add
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < PEAK_CHAINS; ++k) s += x[k];
    out[size_t(blockIdx.x) * 64 + threadIdx.x] = s;
}

}  // namespace

ms_status ms_peak_fp32(float* dev_out, int n_waves, int iters, void* hip_stream) {
    if (!dev_out) return fail(MS_E_INVALID_ARG, "null output");
    if (n_waves <= 0 || iters <= 0) return fail(MS_E_INVALID_ARG, "n_waves and iters must be positive (got %d, %d)", n_waves, iters);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipLaunchKernelGGL(ms_peak_fp32_kernel, dim3(n_waves), dim3(64), 0, s, dev_out, iters, 0.999f, 1e-3f);
    HIP_OK(hipGetLastError());
    return MS_OK;
}
