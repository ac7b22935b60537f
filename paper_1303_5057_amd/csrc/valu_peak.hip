// Vector issue-rate probe for the roofline peaks of the integrators: each
// thread runs 8 independent chains of one operation (FMA, multiply, add, or
// two of them interleaved) in FP32 and FP64, with the other operands in
// scalar or in vector registers, non-packed (built, like the
// library, with packed FP32 disabled), and writes one value. Prints the
// FLOP rate and the SIMD cycles per wave64 instruction (2.4 GHz, 1024 SIMDs).
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o /tmp/valu_peak paper_1303_5057_amd/csrc/valu_peak.hip && /tmp/valu_peak
#include <hip/hip_runtime.h>
#include <cstdio>
#include <vector>
template <typename T, int OP, bool V>
__global__ __launch_bounds__(256) void k_chains(T *out, int iters, T bs, T cs)
{
    // V: the multiplier and addend in vector registers (per-lane values),
    // else in scalar registers (kernel arguments)
    const T b = V ? bs + (T)threadIdx.x * (T)1e-9 : bs;
    const T c = V ? cs + (T)threadIdx.x * (T)1e-9 : cs;
    T a0 = (T)threadIdx.x * (T)1e-3, a1 = a0 + (T)1, a2 = a0 + (T)2, a3 = a0 + (T)3;
    T a4 = a0 + (T)4, a5 = a0 + (T)5, a6 = a0 + (T)6, a7 = a0 + (T)7;
    for (int i = 0; i < iters; ++i) {
        if constexpr (OP == 0) {
            a0 = fma(a0, b, c); a1 = fma(a1, b, c); a2 = fma(a2, b, c); a3 = fma(a3, b, c);
            a4 = fma(a4, b, c); a5 = fma(a5, b, c); a6 = fma(a6, b, c); a7 = fma(a7, b, c);
        } else if constexpr (OP == 1) {
            a0 = a0 * b; a1 = a1 * b; a2 = a2 * b; a3 = a3 * b;
            a4 = a4 * b; a5 = a5 * b; a6 = a6 * b; a7 = a7 * b;
        } else if constexpr (OP == 2) {
            a0 = a0 + c; a1 = a1 + c; a2 = a2 + c; a3 = a3 + c;
            a4 = a4 + c; a5 = a5 + c; a6 = a6 + c; a7 = a7 + c;
        } else if constexpr (OP == 3) {   // fma and mul interleaved
            a0 = fma(a0, b, c); a1 = a1 * b; a2 = fma(a2, b, c); a3 = a3 * b;
            a4 = fma(a4, b, c); a5 = a5 * b; a6 = fma(a6, b, c); a7 = a7 * b;
        } else if constexpr (OP == 4) {   // fma and add interleaved
            a0 = fma(a0, b, c); a1 = a1 + c; a2 = fma(a2, b, c); a3 = a3 + c;
            a4 = fma(a4, b, c); a5 = a5 + c; a6 = fma(a6, b, c); a7 = a7 + c;
        } else {                          // mul and add interleaved
            a0 = a0 * b; a1 = a1 + c; a2 = a2 * b; a3 = a3 + c;
            a4 = a4 * b; a5 = a5 + c; a6 = a6 * b; a7 = a7 + c;
        }
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
}
template <typename T, int OP, bool V = false>
double run(const char *name, int blocks, int iters)
{
    T *out;
    const size_t n = (size_t)blocks * 256;
    if (hipMalloc(&out, n * sizeof(T)) != hipSuccess) { printf("alloc failed\n"); return 0; }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) { printf("event failed\n"); return 0; }
    float best = 1e30f;
    for (int r = 0; r < 6; ++r) {
        float ms = 0.0f;
        bool ok = hipEventRecord(e0, 0) == hipSuccess;
        hipLaunchKernelGGL((k_chains<T, OP, V>), dim3(blocks), dim3(256), 0, 0, out, iters, (T)0.999, (T)1e-3);
        ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, 0) == hipSuccess;
        ok = ok && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) { printf("launch or timing failed\n"); return 0; }
        if (r > 0 && ms < best) best = ms;
    }
    std::vector<T> h(4);
    if (hipMemcpy(h.data(), out, 4 * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) printf("copy failed\n");
    const double insts = (double)n / 64 * iters * 8;   // wave-level instructions
    const double flops = (double)n * iters * (OP == 0 ? 16 : (OP == 3 || OP == 4) ? 12 : 8);
    printf("%s blocks %d iters %d: %.3f ms, %.1f TFLOP/s, %.2f SIMD-cycles per wave instruction (check %g)\n", name, blocks,
           iters, best, flops / best / 1e9, best * 1e-3 * 2.4e9 * 1024 / insts, (double)h[0]);
    (void)hipFree(out);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return flops / best / 1e9;
}
int main()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) return 1;
    printf("%s CUs %d clock %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
    const int blocks = 16384;
    run<float, 0>("fp32 fma", blocks, 4096);
    run<float, 1>("fp32 mul", blocks, 4096);
    run<float, 2>("fp32 add", blocks, 4096);
    run<float, 3>("fp32 fma+mul", blocks, 4096);
    run<float, 4>("fp32 fma+add", blocks, 4096);
    run<float, 5>("fp32 mul+add", blocks, 4096);
    run<double, 0>("fp64 fma", blocks, 4096);
    run<double, 1>("fp64 mul", blocks, 4096);
    run<double, 2>("fp64 add", blocks, 4096);
    run<double, 3>("fp64 fma+mul", blocks, 4096);
    run<double, 4>("fp64 fma+add", blocks, 4096);
    run<double, 5>("fp64 mul+add", blocks, 4096);
    run<float, 0, true>("fp32 fma, vector operands", blocks, 4096);
    run<float, 1, true>("fp32 mul, vector operands", blocks, 4096);
    run<float, 3, true>("fp32 fma+mul, vector operands", blocks, 4096);
    run<double, 0, true>("fp64 fma, vector operands", blocks, 4096);
    run<double, 1, true>("fp64 mul, vector operands", blocks, 4096);
    return 0;
}
