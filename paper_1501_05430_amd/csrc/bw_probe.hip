// Bandwidth probes for the benchmark (not part of the method's library): the ceilings the step kernel is held
// against on the GPU it runs on.
//  * bwp_copy: a streaming copy of float4 (or float) elements, src -> dst, each thread moving UNROLL elements with a
//    stride of the block size so every wavefront touches whole 1 KiB (float4) runs. Read + write bytes count.
//  * bwp_pattern: the step kernel's memory pattern with no arithmetic: population planes [9][ny-2][pitch] (FP32),
//    blocks of 512 columns x a strip of rows walking upwards (or downwards), each lane gathering the nine pulled
//    populations of its column (x - e_i, y - e_i, x periodic, the wall rows bouncing back) plus the block's two halo
//    columns, one row ahead of the store of the previous row. It shows what the step kernel's access pattern
//    achieves when nothing else limits it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kCopyBlock = 256;
constexpr int kUnroll = 4;

template <class V>
__global__ __launch_bounds__(kCopyBlock) void k_copy(const V* __restrict__ src, V* __restrict__ dst, size_t n) {
  const size_t base = (size_t)blockIdx.x * (kCopyBlock * kUnroll) + threadIdx.x;
  V v[kUnroll];
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const size_t i = base + (size_t)u * kCopyBlock;
    if (i < n) v[u] = src[i];
  }
#pragma unroll
  for (int u = 0; u < kUnroll; ++u) {
    const size_t i = base + (size_t)u * kCopyBlock;
    if (i < n) dst[i] = v[u];
  }
}

constexpr int kPatWaves = 8;
constexpr int kPatCols = 64 * kPatWaves;
__device__ constexpr int kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__device__ constexpr int kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// The nine pulled populations of fluid node (x, y) (rows 1..ny-2), summed: the same addresses the step reads.
__device__ inline float pulled_sum(const float* __restrict__ g, int64_t plane, int pitch, int nx, int ny, int x,
                                   int y) {
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = x - kEX[i], ys = y - kEY[i];
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    int q = i;
    if (ys < 1 || ys > ny - 2) {  // halfway bounce-back: the node's own opposite population
      ys = y;
      xs = x;
      q = kOPP[i];
    }
    s += g[q * plane + (int64_t)(ys - 1) * pitch + xs];
  }
  return s;
}

__global__ __launch_bounds__(kPatCols) void k_pattern(const float* __restrict__ gin, float* __restrict__ gout,
                                                      int nx, int ny, int pitch, int strip_rows, int down) {
  const int nyf = ny - 2;
  const int nbx = (nx + kPatCols - 1) / kPatCols;
  const int bx = (int)blockIdx.x % nbx, by = (int)blockIdx.x / nbx;
  const int x0 = bx * kPatCols;
  const int y0 = 1 + by * strip_rows;
  const int y1 = min(y0 + strip_rows, ny - 1);  // exclusive
  const int lx = (int)threadIdx.x;
  const bool act = x0 + lx < nx;
  const int x = act ? x0 + lx : x0;
  const int bw = min(kPatCols, nx - x0);
  const bool edge = lx == 0 || lx == bw - 1;
  const int hx = lx == 0 ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + bw == nx ? 0 : x0 + bw);
  const int64_t plane = (int64_t)nyf * pitch;
  const int st = down ? -1 : 1;
  const int ya = down ? y1 - 1 : y0, yb = down ? y0 : y1 - 1;
  // rows gathered: one beyond each end of the strip (the force's neighbour rows), within the fluid rows
  const int ylo = max(y0 - 1, 1), yhi = min(y1, ny - 2);
  float acc = 0.0f;
  float cur = 0.0f;
  auto gathered = [&](int y) -> float {
    if (y < ylo || y > yhi) return 0.0f;
    float v = act ? pulled_sum(gin, plane, pitch, nx, ny, x, y) : 0.0f;
    if (edge) v += pulled_sum(gin, plane, pitch, nx, ny, hx, y);
    return v;
  };
  float behind = gathered(ya - st);
  cur = gathered(ya);
  for (int y = ya;; y += st) {
    const float ahead = gathered(y + st);
    acc = behind + cur + ahead;
    if (act) {
      const int64_t off = (int64_t)(y - 1) * pitch + x;
#pragma unroll
      for (int i = 0; i < 9; ++i) gout[i * plane + off] = acc * (float)(i + 1);
    }
    if (y == yb) break;
    behind = cur;
    cur = ahead;
  }
}

int status(hipError_t e) { return e == hipSuccess ? 0 : (int)e; }

}  // namespace

extern "C" {

// Copy `bytes` bytes from src to dst on the stream (vec = 4: float4 elements, bytes a multiple of 16; vec = 1:
// float elements, a multiple of 4). Returns 0 or the hipError_t of the launch; 1 on bad arguments.
int bwp_copy(const void* src, void* dst, size_t bytes, int vec, void* stream) {
  if (!src || !dst || (vec != 1 && vec != 4) || bytes % (4 * (size_t)vec) != 0) return 1;
  const size_t n = bytes / (4 * (size_t)vec);
  if (n == 0) return 0;
  const size_t blocks = (n + kCopyBlock * kUnroll - 1) / (kCopyBlock * kUnroll);
  if (vec == 4)
    hipLaunchKernelGGL(k_copy<float4>, dim3((unsigned)blocks), dim3(kCopyBlock), 0, (hipStream_t)stream,
                       (const float4*)src, (float4*)dst, n);
  else
    hipLaunchKernelGGL(k_copy<float>, dim3((unsigned)blocks), dim3(kCopyBlock), 0, (hipStream_t)stream,
                       (const float*)src, (float*)dst, n);
  return status(hipGetLastError());
}

// The step's memory pattern over FP32 planes [9][ny-2][pitch] (gin read, gout written; pitch >= nx, a multiple of
// 64), strips of strip_rows rows, walking downwards when down != 0. Returns 0, a hipError_t, or 1 on bad arguments.
int bwp_pattern(const float* gin, float* gout, int nx, int ny, int pitch, int strip_rows, int down, void* stream) {
  if (!gin || !gout || nx < 2 || ny < 4 || pitch < nx || pitch % 64 != 0 || strip_rows < 1) return 1;
  const int nbx = (nx + kPatCols - 1) / kPatCols;
  const int nby = (ny - 2 + strip_rows - 1) / strip_rows;
  hipLaunchKernelGGL(k_pattern, dim3((unsigned)(nbx * nby)), dim3(kPatCols), 0, (hipStream_t)stream, gin, gout, nx,
                     ny, pitch, strip_rows, down);
  return status(hipGetLastError());
}

}  // extern "C"
