// Reference bandwidth of the step's memory traffic without its arithmetic.
//
//     hbm_ceiling [nx ny iterations]
//
// Times, on an nx x ny lattice in the row-interleaved population layout of
// the step (row y holds the nine population rows of lattice row y, each px
// elements), a kernel that reads the nine population rows of every lattice
// row and writes them to a second buffer with non-temporal stores, in FP64
// and in FP32, plus a plain vectorised copy of the same number of bytes.
// As checks on those figures from other access patterns it also times a
// read-only stream of the FP64 buffer (32-byte loads, nothing stored), a
// write-only stream of it (32-byte stores), and the runtime's own
// device-to-device copy of it (hipMemcpyAsync).  Prints one JSON line.  A
// step that moves 144 (72) bytes per node cannot run faster than the first
// two figures allow.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                               \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) {                                                    \
      fprintf(stderr, "hbm_ceiling: %s: %s\n", #x, hipGetErrorString(e_));    \
      exit(1);                                                                 \
    }                                                                          \
  } while (0)

namespace {

constexpr int Q = 9;

// One block per strip of BW columns and chunk of `rows` lattice rows; each
// thread streams its column, D rows of populations in flight.
template <typename T, int BW, int D>
__global__ void __launch_bounds__(BW)
    rows_copy(const T* __restrict__ fin, T* __restrict__ fout, int px, int ny, int rows, int strips) {
  const int strip = blockIdx.x % strips, chunk = blockIdx.x / strips;
  const int x = strip * BW + threadIdx.x;
  const long long pitch = (long long)Q * px;
  const int y0 = chunk * rows;
  const int H = min(rows, ny - y0);
  T buf[D + 1][Q];
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < H)
#pragma unroll
      for (int q = 0; q < Q; ++q) buf[d][q] = fin[(y0 + d) * pitch + (long long)q * px + x];
  for (int k = 0; k < H; k += D + 1) {
#pragma unroll
    for (int s = 0; s <= D; ++s) {
      const int r = k + s, l = r + D, sl = (s + D) % (D + 1);
      if (l < H)
#pragma unroll
        for (int q = 0; q < Q; ++q) buf[sl][q] = fin[(y0 + l) * pitch + (long long)q * px + x];
      if (r < H)
#pragma unroll
        for (int q = 0; q < Q; ++q)
          __builtin_nontemporal_store(buf[s][q], &fout[(y0 + r) * pitch + (long long)q * px + x]);
    }
  }
}

__global__ void copy_vec(const double4* __restrict__ a, double4* __restrict__ b, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// Reads every element; the store is taken only for a sum no buffer of this
// program holds (the buffers are zero), so nothing is written, but the
// loads cannot be dropped.
__global__ void read_vec(const double4* __restrict__ a, double* __restrict__ out, long long n) {
  double s = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double4 v = a[i];
    s += (v.x + v.y) + (v.z + v.w);
  }
  if (s == 1234.5) out[blockIdx.x] = s;
}

__global__ void write_vec(double4* __restrict__ b, long long n) {
  const double4 z = make_double4(0.0, 0.0, 0.0, 0.0);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    b[i] = z;
}

template <typename F>
double time_us(F launch, int iters, hipEvent_t e0, hipEvent_t e1) {
  launch();
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0));
  for (int i = 0; i < iters; ++i) launch();
  CHECK(hipEventRecord(e1));
  CHECK(hipEventSynchronize(e1));
  float ms = 0;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return 1e3 * ms / iters;
}

}  // namespace

int main(int argc, char** argv) {
  const int nx = argc > 1 ? atoi(argv[1]) : 4096;
  const int ny = argc > 2 ? atoi(argv[2]) : 4096;
  const int iters = argc > 3 ? atoi(argv[3]) : 20;
  constexpr int BW = 512, D = 1, ROWS = 128;
  if (nx < BW || nx % BW || ny < 1 || iters < 1) {
    fprintf(stderr, "hbm_ceiling: nx must be a positive multiple of %d, ny and iterations positive\n", BW);
    return 2;
  }
  const int px = nx;
  const long long elems = (long long)Q * px * ny;  // per buffer
  const size_t bytes = (size_t)elems * sizeof(double);
  void *a = nullptr, *b = nullptr;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMemset(a, 0, bytes));
  CHECK(hipMemset(b, 0, bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int strips = nx / BW, chunks = (ny + ROWS - 1) / ROWS;
  const double us64 = time_us([&] {
    rows_copy<double, BW, D><<<strips * chunks, BW>>>((const double*)a, (double*)b, px, ny, ROWS, strips);
  }, iters, e0, e1);
  const double us32 = time_us([&] {
    rows_copy<float, BW, D><<<strips * chunks, BW>>>((const float*)a, (float*)b, px, ny, ROWS, strips);
  }, iters, e0, e1);
  const long long n4 = elems / 4;  // double4 elements of one FP64 buffer
  const double usc = time_us([&] {
    copy_vec<<<65536, 256>>>((const double4*)a, (double4*)b, n4);
  }, iters, e0, e1);
  double* sink = nullptr;
  CHECK(hipMalloc(&sink, 65536 * sizeof(double)));
  const double usr = time_us([&] {
    read_vec<<<65536, 256>>>((const double4*)a, sink, n4);
  }, iters, e0, e1);
  const double usw = time_us([&] { write_vec<<<65536, 256>>>((double4*)b, n4); }, iters, e0, e1);
  const double usd = time_us([&] {
    CHECK(hipMemcpyAsync(b, a, bytes, hipMemcpyDeviceToDevice, 0));
  }, iters, e0, e1);
  CHECK(hipGetLastError());
  const double nodes = (double)nx * ny;
  printf("{\"nx\": %d, \"ny\": %d, \"rows_copy_fp64_us\": %.1f, \"rows_copy_fp64_gbs\": %.0f, "
         "\"rows_copy_fp32_us\": %.1f, \"rows_copy_fp32_gbs\": %.0f, \"vector_copy_gbs\": %.0f, "
         "\"read_only_gbs\": %.0f, \"write_only_gbs\": %.0f, \"runtime_d2d_copy_gbs\": %.0f, "
         "\"buffer_bytes\": %zu}\n",
         nx, ny, us64, 144.0 * nodes / us64 / 1e3, us32, 72.0 * nodes / us32 / 1e3,
         2.0 * bytes / usc / 1e3, bytes / usr / 1e3, bytes / usw / 1e3, 2.0 * bytes / usd / 1e3,
         bytes);
  CHECK(hipFree(sink));
  CHECK(hipFree(a));
  CHECK(hipFree(b));
  return 0;
}
