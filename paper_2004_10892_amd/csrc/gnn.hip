// Learned proposal: a message-passing network over the variables of a
// (reduced) graphical model, trained on the device.
//
// Architecture (fixed): input features F = 8 per variable, three layers of
//   H_{l+1} = relu(H_l W_s + mean_{w in N(v)} H_l[w] W_n + b)      (width 64)
// shared by two linear heads s_h = H_3 w_h + c_h: head 0 scores variables
// for slicing (Alg. 2), head 1 for elimination (ties of greedy min-fill).
// The dense layers and their gradients run on MFMA (v_mfma_f32_16x16x4f32:
// FP32 activations times the FP16 weights widened exactly to FP32).
// Weights are FP16 in the forward and
// backward passes (FP32 master copies for the optimizer); every sum is
// accumulated in FP32.  Training minimises the mean squared error between s
// and a target at a set of candidate variables.  All reductions run in a
// fixed order (no atomics): the same inputs give the same bits.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/qbe.h"
#include "qbe_internal.hpp"

namespace qbe {

#define GNN_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      set_error(std::string(#call) + ": " + hipGetErrorString(e_));                     \
      return QBE_ERR_HIP;                                                               \
    }                                                                                   \
  } while (0)

// ------------------------------------------------------------- parameters --
// Flat parameter vector: for layer l = 0..2 (din = 8, 64, 64):
//   W_s[din][64], W_n[din][64], b[64]; then head 0 (w[64], c), head 1 (w[64], c).
__host__ __device__ constexpr int gnn_din(int l) { return l == 0 ? kGnnFeatures : kGnnHidden; }
__host__ __device__ constexpr int gnn_layer_size(int l) { return 2 * gnn_din(l) * kGnnHidden + kGnnHidden; }
__host__ __device__ constexpr int gnn_layer_off(int l) {
  return l == 0 ? 0 : gnn_layer_off(l - 1) + gnn_layer_size(l - 1);
}
constexpr int kGnnHeadOff = gnn_layer_off(kGnnLayers);
constexpr int kGnnHeadSize = kGnnHidden + 1;
constexpr int kGnnParams = kGnnHeadOff + kGnnHeads * kGnnHeadSize;

int gnn_num_params() { return kGnnParams; }
static_assert(kGnnFeatures == kFeatures, "feature width");

// ---------------------------------------------------------------- kernels --

// M[v][d] = mean over neighbours w of H[w][d] (0 for an isolated vertex).
__global__ void gnn_agg(const float* __restrict__ H, const int* __restrict__ rp, const int* __restrict__ col,
                        int n, int D, float* __restrict__ M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * D) return;
  const int v = (int)(i / D), d = (int)(i % D);
  const int b = rp[v], e = rp[v + 1];
  float s = 0.f;
  for (int j = b; j < e; ++j) s += H[(int64_t)col[j] * D + d];
  M[i] = e > b ? s / (float)(e - b) : 0.f;
}

// dH[w][d] = dHs[w][d] + sum over neighbours v of dM[v][d] / deg(v)
// (the transpose of gnn_agg on the symmetric adjacency).
__global__ void gnn_agg_t(const float* __restrict__ dHs, const float* __restrict__ dM, const int* __restrict__ rp,
                          const int* __restrict__ col, int n, int D, float* __restrict__ dH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * D) return;
  const int w = (int)(i / D), d = (int)(i % D);
  float s = dHs[i];
  for (int j = rp[w]; j < rp[w + 1]; ++j) {
    const int v = col[j];
    s += dM[(int64_t)v * D + d] / (float)(rp[v + 1] - rp[v]);
  }
  dH[i] = s;
}

// The dense layer as matrix products on MFMA: [H | M] (n x 2 din, FP32)
// times [Ws ; Wn] (2 din x 64, the FP16 weights widened to FP32 -- exact),
// v_mfma_f32_16x16x4f32 with FP32 accumulation.  A workgroup takes 16
// vertices and each of its four waves one 16 x 16 tile of the 64 outputs,
// accumulated over K in steps of 4; the weights are read straight from the
// (cached) FP16 copy, so every workgroup starts at once and a layer of n
// vertices runs n / 16 of them.  Lane l supplies A[row l % 16][k = l / 16]
// and B[k][col l % 16] and receives C[4 (l / 16) + j][l % 16], j = 0..3
// (the layout mm_kernel uses).
typedef float gnn_f4 __attribute__((ext_vector_type(4)));
constexpr int kGnnRows = 16;  // vertices per workgroup

__global__ __launch_bounds__(256) void gnn_dense_mfma(const float* __restrict__ Hin, const float* __restrict__ Min,
                                                      const __half* __restrict__ w, int din, int n,
                                                      float* __restrict__ Z, float* __restrict__ Hout) {
  const int tid = threadIdx.x, lane = tid & 63, row = lane & 15, grp = lane >> 4, c = tid >> 6;
  const int v0 = blockIdx.x * kGnnRows;
  const int vr = v0 + row;
  const bool ok = vr < n;
  gnn_f4 acc = gnn_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
  for (int kb = 0; kb < 2 * din; kb += 4) {
    const int k = kb + grp;
    const float a = ok ? (k < din ? Hin[(int64_t)vr * din + k] : Min[(int64_t)vr * din + (k - din)]) : 0.f;
    const float b = __half2float(w[k * kGnnHidden + c * 16 + row]);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  const int o = c * 16 + row;
  const float bias = __half2float(w[2 * din * kGnnHidden + o]);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int v = v0 + 4 * grp + j;
    if (v >= n) continue;
    const float z = acc[j] + bias;
    Z[(int64_t)v * kGnnHidden + o] = z;
    Hout[(int64_t)v * kGnnHidden + o] = z > 0.f ? z : 0.f;
  }
}

// dHs = dZ Ws^T and dM = dZ Wn^T (din = 64) on MFMA: A = dZ (n x 64), B[o][k]
// = the weight of input k to output o.  A workgroup takes 16 vertices x 128
// columns (64 of dHs, 64 of dM) in eight 16 x 16 tiles, two per wave; the
// weights are read from the FP16 copy as in the forward.
__global__ __launch_bounds__(256) void gnn_dense_back_x_mfma(const float* __restrict__ dZ,
                                                             const __half* __restrict__ w, int n,
                                                             float* __restrict__ dHs, float* __restrict__ dM) {
  const int tid = threadIdx.x, lane = tid & 63, row = lane & 15, grp = lane >> 4, c0 = 2 * (tid >> 6);
  const int v0 = blockIdx.x * kGnnRows;
  const int vr = v0 + row;
  const bool ok = vr < n;
  gnn_f4 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) acc[t] = gnn_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int ob = 0; ob < kGnnHidden; ob += 4) {
    const int o = ob + grp;
    const float a = ok ? dZ[(int64_t)vr * kGnnHidden + o] : 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      // column c * 16 + row: input k of Ws (c < 4) or of Wn (c >= 4)
      const int c = c0 + t, k = (c & 3) * 16 + row;
      const float b = __half2float(w[((c >> 2) * kGnnHidden + k) * kGnnHidden + o]);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int v = v0 + 4 * grp + j;
      if (v >= n) continue;
      const int c = c0 + t, k = (c & 3) * 16 + row;
      (c < 4 ? dHs : dM)[(int64_t)v * kGnnHidden + k] = acc[t][j];
    }
}

__global__ void gnn_head(const float* __restrict__ H, const __half* __restrict__ w, int n, float* __restrict__ s) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  float a = __half2float(w[kGnnHidden]);
  for (int o = 0; o < kGnnHidden; ++o) a += H[(int64_t)v * kGnnHidden + o] * __half2float(w[o]);
  s[v] = a;
}

// dS = 0 except at the candidates: 2 (s - y) / n_c; loss = mean (s - y)^2.
// One block, candidates in a fixed order.
__global__ void gnn_loss(const float* __restrict__ s, const int* __restrict__ cand, const float* __restrict__ y,
                         int nc, int n, float* __restrict__ dS, float* __restrict__ loss) {
  __shared__ float part[256];
  for (int v = threadIdx.x; v < n; v += blockDim.x) dS[v] = 0.f;
  __syncthreads();
  float acc = 0.f;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) {
    const float d = s[cand[i]] - y[i];
    dS[cand[i]] = 2.f * d / (float)nc;
    acc += d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = part[0] / (float)(nc > 0 ? nc : 1);
}

// Head backward: dH[v][o] = dS[v] w[o] (its weight gradient: gnn_head_back_w_part).
__global__ void gnn_head_back_x(const float* __restrict__ dS, const __half* __restrict__ w, int n,
                                float* __restrict__ dH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * kGnnHidden) return;
  dH[i] = dS[i / kGnnHidden] * __half2float(w[i % kGnnHidden]);
}

// dZ = dH * (Z > 0), in place into dH.
__global__ void gnn_relu_back(float* __restrict__ dH, const float* __restrict__ Z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(Z[i] > 0.f)) dH[i] = 0.f;
}

// Weight gradients are sums over all vertices.  They run in two passes
// with a fixed order: every workgroup sums one chunk of kGnnChunk vertices
// into a partial, then gnn_sum_parts adds the partials in chunk order.
constexpr int kGnnChunk = 64;

// Partial of layer l's gradient over chunk blockIdx.x: row k of [Ws ; Wn]
// (input k of H for k < din, of M after), P[k][o] = sum_v X[v][k] dZ[v][o]
// on MFMA (A = a 16 x 4 tile of X^T, B = a 4 x 16 tile of dZ, vertices as
// the contraction), and the bias row P[2 din][o] = sum_v dZ[v][o].  The
// (2 din / 16) x 4 tiles of 16 x 16 go one to a wave, four to a workgroup
// along blockIdx.y (a chunk's tiles run side by side, not one after another
// in a wave); the bias row is summed by the blockIdx.y = 0 workgroup.
__global__ __launch_bounds__(256) void gnn_dense_back_w_part(const float* __restrict__ Hin,
                                                             const float* __restrict__ Min,
                                                             const float* __restrict__ dZ, int din, int n,
                                                             float* __restrict__ part) {
  const int tid = threadIdx.x, lane = tid & 63, row = lane & 15, grp = lane >> 4;
  const int vb0 = blockIdx.x * kGnnChunk, ve = min(n, vb0 + kGnnChunk);
  const int rows = 2 * din, len = (rows + 1) * kGnnHidden;
  float* P = part + (int64_t)blockIdx.x * len;
  const int tile = (int)blockIdx.y * 4 + (tid >> 6);
  if (tile < (rows / 16) * 4) {
    const int rt = tile >> 2, ct = tile & 3;
    const int k = rt * 16 + row;
    gnn_f4 acc = gnn_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int vb = vb0; vb < ve; vb += 4) {
      const int v = vb + grp;
      const bool ok = v < ve;
      const float a = ok ? (k < din ? Hin[(int64_t)v * din + k] : Min[(int64_t)v * din + (k - din)]) : 0.f;
      const float b = ok ? dZ[(int64_t)v * kGnnHidden + ct * 16 + row] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) P[(rt * 16 + 4 * grp + j) * kGnnHidden + ct * 16 + row] = acc[j];
  }
  if (blockIdx.y == 0 && tid < kGnnHidden) {
    float sb = 0.f;
#pragma unroll 8
    for (int v = vb0; v < ve; ++v) sb += dZ[(int64_t)v * kGnnHidden + tid];
    P[rows * kGnnHidden + tid] = sb;
  }
}

// Partial of a head's gradient over one chunk: g_w[o] = sum_v dS[v] H[v][o]
// (o < 64), g_c = sum_v dS[v] (o = 64).
__global__ __launch_bounds__(128) void gnn_head_back_w_part(const float* __restrict__ dS,
                                                            const float* __restrict__ H, int n,
                                                            float* __restrict__ part) {
  const int o = threadIdx.x;
  if (o > kGnnHidden) return;
  const int vb0 = blockIdx.x * kGnnChunk, ve = min(n, vb0 + kGnnChunk);
  float a = 0.f;
#pragma unroll 8
  for (int v = vb0; v < ve; ++v) a += dS[v] * (o < kGnnHidden ? H[(int64_t)v * kGnnHidden + o] : 1.f);
  part[(int64_t)blockIdx.x * (kGnnHidden + 1) + o] = a;
}

// g[i] = sum over the n_parts partials (chunk order) of entry i.
__global__ void gnn_sum_parts(const float* __restrict__ part, int n_parts, int len, float* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  float a = 0.f;
#pragma unroll 8
  for (int c = 0; c < n_parts; ++c) a += part[(int64_t)c * len + i];
  g[i] = a;
}

// Adam on the FP32 master weights, refreshing the FP16 copy.
__global__ void gnn_adam(float* __restrict__ p, __half* __restrict__ p16, const float* __restrict__ g,
                         float* __restrict__ m, float* __restrict__ v, int n, float lr, float b1, float b2,
                         float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  p16[i] = __float2half(pi);
}

__global__ void gnn_zero(float* __restrict__ x, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0.f;
}

__global__ void gnn_to_half(const float* __restrict__ p, __half* __restrict__ p16, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p16[i] = __float2half(p[i]);
}

// ------------------------------------------------------------------- host --

static unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int gnn_alloc(Gnn& g, int device) {
  g.device = device;
  GNN_HIP(hipMalloc(&g.d_p, kGnnParams * 4));
  GNN_HIP(hipMalloc(&g.d_p16, kGnnParams * 2));
  GNN_HIP(hipMalloc(&g.d_g, kGnnParams * 4));
  GNN_HIP(hipMalloc(&g.d_m, kGnnParams * 4));
  GNN_HIP(hipMalloc(&g.d_v, kGnnParams * 4));
  GNN_HIP(hipMemset(g.d_m, 0, kGnnParams * 4));
  GNN_HIP(hipMemset(g.d_v, 0, kGnnParams * 4));
  g.step = 0;
  return QBE_OK;
}

void gnn_free(Gnn& g) {
  void** ptrs[] = {&g.d_p, &g.d_p16, &g.d_g, &g.d_m, &g.d_v, &g.d_ws};
  for (void** q : ptrs) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  g.ws_bytes = 0;
}

int gnn_set_params(Gnn& g, const float* host, bool reset_optimizer) {
  GNN_HIP(hipMemcpy(g.d_p, host, kGnnParams * 4, hipMemcpyHostToDevice));
  gnn_to_half<<<blocks(kGnnParams), 256>>>((const float*)g.d_p, (__half*)g.d_p16, kGnnParams);
  GNN_HIP(hipGetLastError());
  if (reset_optimizer) {
    GNN_HIP(hipMemset(g.d_m, 0, kGnnParams * 4));
    GNN_HIP(hipMemset(g.d_v, 0, kGnnParams * 4));
    g.step = 0;
  }
  GNN_HIP(hipDeviceSynchronize());
  return QBE_OK;
}

int gnn_get_params(const Gnn& g, float* host) {
  GNN_HIP(hipMemcpy(host, g.d_p, kGnnParams * 4, hipMemcpyDeviceToHost));
  return QBE_OK;
}

int gnn_get_state(const Gnn& g, float* p, float* m, float* v, int* step) {
  GNN_HIP(hipMemcpy(p, g.d_p, kGnnParams * 4, hipMemcpyDeviceToHost));
  GNN_HIP(hipMemcpy(m, g.d_m, kGnnParams * 4, hipMemcpyDeviceToHost));
  GNN_HIP(hipMemcpy(v, g.d_v, kGnnParams * 4, hipMemcpyDeviceToHost));
  *step = g.step;
  return QBE_OK;
}

int gnn_set_state(Gnn& g, const float* p, const float* m, const float* v, int step) {
  int rc = gnn_set_params(g, p, false);
  if (rc) return rc;
  GNN_HIP(hipMemcpy(g.d_m, m, kGnnParams * 4, hipMemcpyHostToDevice));
  GNN_HIP(hipMemcpy(g.d_v, v, kGnnParams * 4, hipMemcpyHostToDevice));
  g.step = step;
  return QBE_OK;
}

// Device workspace for a graph of n vertices and nnz adjacency entries, the
// candidates, and every activation the backward pass needs.
struct GnnBufs {
  int *rp, *col, *cand;
  float *X, *y, *s, *dS, *loss;
  float* H[kGnnLayers + 1];
  float* M[kGnnLayers];
  float* Z[kGnnLayers];
  float *dA, *dB, *dC;  // backward scratch (n x 64 each)
  float* part;          // weight-gradient partials, one per chunk of vertices
};

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

static int gnn_layout(Gnn& g, int n, int64_t nnz, int nc, GnnBufs& b) {
  const size_t sizes[] = {
      (size_t)(n + 1) * 4, (size_t)nnz * 4, (size_t)nc * 4,                 // rp, col, cand
      (size_t)n * kGnnFeatures * 4, (size_t)nc * 4, (size_t)n * 4, (size_t)n * 4, 256,  // X, y, s, dS, loss
  };
  size_t need = 0;
  for (size_t z : sizes) need += align256(z);
  need += kGnnLayers * align256((size_t)n * kGnnHidden * 4);        // H[1..L]
  need += kGnnLayers * align256((size_t)n * kGnnHidden * 4) * 2;    // M, Z (M[0] sized for 64 too)
  need += 3 * align256((size_t)n * kGnnHidden * 4);                  // dA, dB, dC
  const size_t n_parts = ((size_t)n + kGnnChunk - 1) / kGnnChunk;
  need += align256(n_parts * (2 * kGnnHidden + 1) * kGnnHidden * 4);  // partials
  if (need > g.ws_bytes) {
    if (g.d_ws) (void)hipFree(g.d_ws);
    g.d_ws = nullptr;
    g.ws_bytes = 0;
    GNN_HIP(hipMalloc(&g.d_ws, need));
    g.ws_bytes = need;
  }
  char* w = (char*)g.d_ws;
  auto take = [&](size_t bytes) {
    char* p = w;
    w += align256(bytes);
    return p;
  };
  b.rp = (int*)take(sizes[0]);
  b.col = (int*)take(sizes[1]);
  b.cand = (int*)take(sizes[2]);
  b.X = (float*)take(sizes[3]);
  b.y = (float*)take(sizes[4]);
  b.s = (float*)take(sizes[5]);
  b.dS = (float*)take(sizes[6]);
  b.loss = (float*)take(sizes[7]);
  b.H[0] = b.X;
  for (int l = 1; l <= kGnnLayers; ++l) b.H[l] = (float*)take((size_t)n * kGnnHidden * 4);
  for (int l = 0; l < kGnnLayers; ++l) {
    b.M[l] = (float*)take((size_t)n * kGnnHidden * 4);
    b.Z[l] = (float*)take((size_t)n * kGnnHidden * 4);
  }
  b.dA = (float*)take((size_t)n * kGnnHidden * 4);
  b.dB = (float*)take((size_t)n * kGnnHidden * 4);
  b.dC = (float*)take((size_t)n * kGnnHidden * 4);
  b.part = (float*)take(n_parts * (2 * kGnnHidden + 1) * kGnnHidden * 4);
  return QBE_OK;
}

static int gnn_forward(const Gnn& g, const GnnBufs& b, int n, int head, hipStream_t st) {
  const __half* w16 = (const __half*)g.d_p16;
  for (int l = 0; l < kGnnLayers; ++l) {
    const int din = gnn_din(l);
    gnn_agg<<<blocks((int64_t)n * din), 256, 0, st>>>(b.H[l], b.rp, b.col, n, din, b.M[l]);
    gnn_dense_mfma<<<blocks(n, kGnnRows), 256, 0, st>>>(b.H[l], b.M[l], w16 + gnn_layer_off(l), din, n, b.Z[l],
                                                         b.H[l + 1]);
  }
  gnn_head<<<blocks(n), 256, 0, st>>>(b.H[kGnnLayers], w16 + kGnnHeadOff + head * kGnnHeadSize, n, b.s);
  GNN_HIP(hipGetLastError());
  return QBE_OK;
}

static int upload_graph(Gnn& g, GnnBufs& b, int n, const int* rp, const int* col, const float* feats, int nc,
                        const int* cand, const float* y, hipStream_t st) {
  const int64_t nnz = rp[n];
  int rc = gnn_layout(g, n, nnz, nc, b);
  if (rc) return rc;
  GNN_HIP(hipMemcpyAsync(b.rp, rp, (size_t)(n + 1) * 4, hipMemcpyHostToDevice, st));
  if (nnz) GNN_HIP(hipMemcpyAsync(b.col, col, (size_t)nnz * 4, hipMemcpyHostToDevice, st));
  GNN_HIP(hipMemcpyAsync(b.X, feats, (size_t)n * kGnnFeatures * 4, hipMemcpyHostToDevice, st));
  if (nc) {
    GNN_HIP(hipMemcpyAsync(b.cand, cand, (size_t)nc * 4, hipMemcpyHostToDevice, st));
    GNN_HIP(hipMemcpyAsync(b.y, y, (size_t)nc * 4, hipMemcpyHostToDevice, st));
  }
  return QBE_OK;
}

int gnn_score(Gnn& g, void* stream, int head, int n, const int* rp, const int* col, const float* feats,
              float* scores) {
  hipStream_t st = (hipStream_t)stream;
  GnnBufs b{};
  int rc = upload_graph(g, b, n, rp, col, feats, 0, nullptr, nullptr, st);
  if (rc) return rc;
  if ((rc = gnn_forward(g, b, n, head, st))) return rc;
  GNN_HIP(hipMemcpyAsync(scores, b.s, (size_t)n * 4, hipMemcpyDeviceToHost, st));
  GNN_HIP(hipStreamSynchronize(st));
  return QBE_OK;
}

int gnn_train_step(Gnn& g, void* stream, int head, int n, const int* rp, const int* col, const float* feats,
                   int nc, const int* cand, const float* y, float lr, float* loss_out, float* grads_out) {
  hipStream_t st = (hipStream_t)stream;
  GnnBufs b{};
  int rc = upload_graph(g, b, n, rp, col, feats, nc, cand, y, st);
  if (rc) return rc;
  if ((rc = gnn_forward(g, b, n, head, st))) return rc;
  const __half* w16 = (const __half*)g.d_p16;
  float* grad = (float*)g.d_g;
  gnn_loss<<<1, 256, 0, st>>>(b.s, b.cand, b.y, nc, n, b.dS, b.loss);
  // heads: the loss reaches only the scored head; the other's gradient is 0
  const int hoff = kGnnHeadOff + head * kGnnHeadSize;
  gnn_zero<<<1, 256, 0, st>>>(grad + kGnnHeadOff, kGnnHeads * kGnnHeadSize);
  const int n_parts = (n + kGnnChunk - 1) / kGnnChunk;
  gnn_head_back_w_part<<<n_parts, 128, 0, st>>>(b.dS, b.H[kGnnLayers], n, b.part);
  gnn_sum_parts<<<1, 128, 0, st>>>(b.part, n_parts, kGnnHidden + 1, grad + hoff);
  gnn_head_back_x<<<blocks((int64_t)n * kGnnHidden), 256, 0, st>>>(b.dS, w16 + hoff, n, b.dA);
  // layers, last to first; dA holds dH_{l+1}
  float* dH = b.dA;
  float* dHs = b.dB;
  float* dM = b.dC;
  for (int l = kGnnLayers - 1; l >= 0; --l) {
    const int din = gnn_din(l);
    gnn_relu_back<<<blocks((int64_t)n * kGnnHidden), 256, 0, st>>>(dH, b.Z[l], (int64_t)n * kGnnHidden);
    gnn_dense_back_w_part<<<dim3(n_parts, (2 * din / 16 * 4 + 3) / 4), 256, 0, st>>>(b.H[l], b.M[l], dH, din, n,
                                                                                    b.part);
    gnn_sum_parts<<<blocks(gnn_layer_size(l)), 256, 0, st>>>(b.part, n_parts, gnn_layer_size(l),
                                                           grad + gnn_layer_off(l));
    if (l > 0) {
      gnn_dense_back_x_mfma<<<blocks(n, kGnnRows), 256, 0, st>>>(dH, w16 + gnn_layer_off(l), n, dHs, dM);
      // dH_l = dHs + agg^T(dM), written over the dZ buffer (no longer needed)
      gnn_agg_t<<<blocks((int64_t)n * din), 256, 0, st>>>(dHs, dM, b.rp, b.col, n, din, dH);
    }
  }
  GNN_HIP(hipGetLastError());
  if (lr > 0.f) {
    g.step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)g.step), c2 = 1.f - powf(b2, (float)g.step);
    gnn_adam<<<blocks(kGnnParams), 256, 0, st>>>((float*)g.d_p, (__half*)g.d_p16, grad, (float*)g.d_m,
                                                 (float*)g.d_v, kGnnParams, lr, b1, b2, 1e-8f, c1, c2);
    GNN_HIP(hipGetLastError());
  }
  if (loss_out) GNN_HIP(hipMemcpyAsync(loss_out, b.loss, 4, hipMemcpyDeviceToHost, st));
  if (grads_out) GNN_HIP(hipMemcpyAsync(grads_out, grad, kGnnParams * 4, hipMemcpyDeviceToHost, st));
  GNN_HIP(hipStreamSynchronize(st));
  return QBE_OK;
}

}  // namespace qbe
