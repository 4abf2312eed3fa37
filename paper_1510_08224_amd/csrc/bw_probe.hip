// bw_probe.hip -- bandwidth ceilings of the GPU for the step kernel's
// roofline: a plain streaming copy, read-only and write-only streams, and
// the step's 14-plane pull pattern with no arithmetic.  Diagnostic library
// (libbwprobe.so), separate from liblbm.so.
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef float f4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(const f4v* __restrict__ a, f4v* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(a[i], &b[i]);
}

__global__ __launch_bounds__(256) void k_read(const f4v* __restrict__ a, long long n, float* out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    f4v s = {0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) s += a[i];
    const float t = s.x + s.y + s.z + s.w;
    if (t == 12345.678f) out[0] = t;  // keeps the loads; never true for the probe's zero data
}

__global__ __launch_bounds__(256) void k_write(f4v* __restrict__ b, long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const f4v z = {0, 0, 0, 0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(z, &b[i]);
}

// One 16-byte element per thread, no grid-stride loop: the best of the
// copy variants measured on MI355X (more elements per thread, 8- or 4-byte
// elements, non-temporal loads and larger workgroups were all slower).
__global__ __launch_bounds__(256) void k_copy1(const f4v* __restrict__ a, f4v* __restrict__ b) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    __builtin_nontemporal_store(a[i], &b[i]);
}

// dst plane i at (x, y) = src plane i at (x - e_x, y - e_y), interior nodes.
template <class T>
__global__ __launch_bounds__(256) void k_pull14(const T* __restrict__ s, T* __restrict__ d, int nx, int ny,
                                                int pitch, long long plane) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x < 1 || x >= nx - 1 || y < 1 || y >= ny - 1) return;
    const int ex[14] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 1, 0, -1, 0};
    const int ey[14] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 1, 0, -1};
    T v[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) v[i] = s[i * plane + (long long)(y - ey[i]) * pitch + (x - ex[i])];
#pragma unroll
    for (int i = 0; i < 14; ++i) __builtin_nontemporal_store(v[i], &d[i * plane + (long long)y * pitch + x]);
}

// The same pull in the step kernel's row-interleaved layout: population i
// of node (x, y) at y * 14 * row + i * row + x, `row` the padded row length.
template <class T>
__global__ __launch_bounds__(256) void k_pull14_rows(const T* __restrict__ s, T* __restrict__ d, int nx, int ny,
                                                     int row) {
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = blockIdx.y;
    if (x < 1 || x >= nx - 1 || y < 1 || y >= ny - 1) return;
    const int ex[14] = {0, 1, 0, -1, 0, 1, -1, -1, 1, 0, 1, 0, -1, 0};
    const int ey[14] = {0, 0, 1, 0, -1, 1, 1, -1, -1, 0, 0, 1, 0, -1};
    const long long pitch = 14ll * row;
    T v[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) v[i] = s[(long long)(y - ey[i]) * pitch + (long long)i * row + (x - ex[i])];
#pragma unroll
    for (int i = 0; i < 14; ++i) __builtin_nontemporal_store(v[i], &d[(long long)y * pitch + (long long)i * row + x]);
}

extern "C" {
// Each call launches one kernel on `stream` and returns the hipError_t of
// the launch.  Sizes are in bytes (multiples of 16) or nodes.
int bw_copy(const void* a, void* b, long long bytes, int blocks, void* stream) {
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const f4v*)a, (f4v*)b, bytes / 16);
    return (int)hipGetLastError();
}
int bw_read(const void* a, long long bytes, int blocks, float* out, void* stream) {
    hipLaunchKernelGGL(k_read, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const f4v*)a, bytes / 16, out);
    return (int)hipGetLastError();
}
int bw_write(void* b, long long bytes, int blocks, void* stream) {
    hipLaunchKernelGGL(k_write, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (f4v*)b, bytes / 16);
    return (int)hipGetLastError();
}
// bytes: a multiple of 4096 (256 threads of 16 bytes per workgroup).
int bw_copy1(const void* a, void* b, long long bytes, void* stream) {
    if (bytes <= 0 || bytes % 4096) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy1, dim3((unsigned)(bytes / 4096)), dim3(256), 0, (hipStream_t)stream, (const f4v*)a,
                       (f4v*)b);
    return (int)hipGetLastError();
}
// a and b hold ny rows of 14 padded population rows of `row` elements.
int bw_pull14_rows(int elem_bytes, const void* a, void* b, int nx, int ny, int row, void* stream) {
    dim3 g((nx + 255) / 256, ny);
    hipStream_t st = (hipStream_t)stream;
    if (elem_bytes == 8) hipLaunchKernelGGL(k_pull14_rows<double>, g, dim3(256), 0, st, (const double*)a, (double*)b, nx, ny, row);
    else if (elem_bytes == 4) hipLaunchKernelGGL(k_pull14_rows<float>, g, dim3(256), 0, st, (const float*)a, (float*)b, nx, ny, row);
    else if (elem_bytes == 2) hipLaunchKernelGGL(k_pull14_rows<unsigned short>, g, dim3(256), 0, st, (const unsigned short*)a, (unsigned short*)b, nx, ny, row);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}
// a and b hold 14 planes of `plane` elements of `elem_bytes` (8, 4, 2).
int bw_pull14(int elem_bytes, const void* a, void* b, int nx, int ny, int pitch, long long plane, void* stream) {
    dim3 g((nx + 255) / 256, ny);
    hipStream_t st = (hipStream_t)stream;
    if (elem_bytes == 8) hipLaunchKernelGGL(k_pull14<double>, g, dim3(256), 0, st, (const double*)a, (double*)b, nx, ny, pitch, plane);
    else if (elem_bytes == 4) hipLaunchKernelGGL(k_pull14<float>, g, dim3(256), 0, st, (const float*)a, (float*)b, nx, ny, pitch, plane);
    else if (elem_bytes == 2) hipLaunchKernelGGL(k_pull14<unsigned short>, g, dim3(256), 0, st, (const unsigned short*)a, (unsigned short*)b, nx, ny, pitch, plane);
    else return (int)hipErrorInvalidValue;
    return (int)hipGetLastError();
}
}
