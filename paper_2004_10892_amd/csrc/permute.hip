// Bit permutation of tensor indices on gfx950: one tensor's linear index
// re-ordered into another order of its variables.
//
// The contraction kernels of this library read every operand through a bit
// extraction of the bucket's union index instead of re-laying it out, so no
// permute runs on their path; this kernel is the stand-alone operation, for
// callers that need a tensor in another variable order.
//
// Design: a permutation moves input index bit perm[j] to output bit j.  A
// workgroup moves one tile of 2^t entries (t <= 12, 32 KiB of LDS): the tile
// bits are the lowest input bits and the input bits that become the lowest
// output bits, taken alternately while the tile has room, so reads run over
// at least 2^6 contiguous entries (the lowest input bits vary across lanes)
// and so do writes (the lowest output bits vary across lanes).  Every other
// bit is fixed per tile.  Per-lane tile offsets are fixed for the kernel (a
// bit deposit is linear over disjoint bit sets); the per-tile part is a
// scalar loop.  Entries are moved as 64-bit words with non-temporal loads
// and stores (each byte is touched once).  On a 2^28-entry tensor this runs
// at the speed of a device-to-device copy.
#include "device_common.hpp"

#include <vector>

namespace qbe {

namespace {

// Scatter the low bits of v to the set bits of m, lowest first.
__host__ __device__ __forceinline__ uint32_t deposit(uint32_t v, uint32_t m) {
  uint32_t r = 0;
  for (int k = 0; m; ++k, m &= m - 1) r |= ((v >> k) & 1u) << __builtin_ctz(m);
  return r;
}

constexpr int kPermBlock = 512;
constexpr int kPermTileMax = 12;  // tile bits
constexpr int kPermPerThread = (1 << kPermTileMax) / kPermBlock;

struct PermArgs {
  const uint64_t* in;
  uint64_t* out;
  int32_t r, t;
  uint32_t tin, tout;          // tile bits in the input / output index
  uint32_t rin;                // the other input bits
  uint32_t zmap[kPermTileMax]; // output-order tile bit k is input-order tile bit zmap[k]
  int32_t rest_out[32];        // the k-th other input bit (ascending) becomes output bit rest_out[k]
  int64_t n_rest;              // 2^(r - t) tiles per tensor
  int64_t batch;
};

__global__ __launch_bounds__(kPermBlock) void permute_kernel(PermArgs a) {
  __shared__ uint64_t tile[1 << kPermTileMax];
  const int tid = threadIdx.x;
  const int nt = 1 << a.t;
  uint32_t in_off[kPermPerThread], out_off[kPermPerThread], lds_y[kPermPerThread];
#pragma unroll
  for (int j = 0; j < kPermPerThread; ++j) {
    const uint32_t y = (uint32_t)(tid + j * kPermBlock);  // tile index, input order
    in_off[j] = deposit(y, a.tin);
    out_off[j] = deposit(y, a.tout);  // y read as a tile index in output order
    uint32_t yy = 0;
    for (int k = 0; k < a.t; ++k) yy |= ((y >> k) & 1u) << a.zmap[k];
    lds_y[j] = yy;
  }
  const int64_t n_units = a.batch * a.n_rest;
  for (int64_t w = blockIdx.x; w < n_units; w += gridDim.x) {
    const int64_t b = w / a.n_rest;
    const uint32_t rho = (uint32_t)(w - b * a.n_rest);
    const uint32_t rin_part = deposit(rho, a.rin);
    uint32_t rout_part = 0;
    for (int k = 0; k < a.r - a.t; ++k) rout_part |= ((rho >> k) & 1u) << a.rest_out[k];
    const uint64_t* src = a.in + (b << a.r);
    uint64_t* dst = a.out + (b << a.r);
#pragma unroll
    for (int j = 0; j < kPermPerThread; ++j)
      if (tid + j * kPermBlock < nt) tile[tid + j * kPermBlock] = __builtin_nontemporal_load(src + (in_off[j] | rin_part));
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPermPerThread; ++j)
      if (tid + j * kPermBlock < nt) __builtin_nontemporal_store(tile[lds_y[j]], dst + (out_off[j] | rout_part));
    __syncthreads();
  }
}

}  // namespace

int dev_permute(const void* in, void* out, int r, const int32_t* perm, int64_t batch, void* stream) {
  PermArgs a{};
  a.in = (const uint64_t*)in;
  a.out = (uint64_t*)out;
  a.r = r;
  a.batch = batch;
  // tile bits: the next lowest input bit and the input bit of the next
  // lowest output bit, alternately, while they fit
  a.tin = 0;
  int kin = 0, kout = 0;
  for (bool grew = true; grew;) {
    grew = false;
    if (kin < r && __builtin_popcount(a.tin | (1u << kin)) <= kPermTileMax) {
      a.tin |= 1u << kin++;
      grew = true;
    }
    if (kout < r && __builtin_popcount(a.tin | (1u << perm[kout])) <= kPermTileMax) {
      a.tin |= 1u << perm[kout++];
      grew = true;
    }
  }
  a.t = __builtin_popcount(a.tin);
  std::vector<int> out_of(r);  // output bit j holds input bit perm[j]
  for (int j = 0; j < r; ++j) out_of[perm[j]] = j;
  a.tout = 0;
  for (int p = 0; p < r; ++p)
    if ((a.tin >> p) & 1u) a.tout |= 1u << out_of[p];
  std::vector<int> rank_in(r, -1);  // rank of each tile input bit within tin
  int c = 0;
  for (int p = 0; p < r; ++p)
    if ((a.tin >> p) & 1u) rank_in[p] = c++;
  c = 0;
  for (int j = 0; j < r; ++j)
    if ((a.tout >> j) & 1u) a.zmap[c++] = (uint32_t)rank_in[perm[j]];
  a.rin = (uint32_t)((uint64_t(1) << r) - 1u) & ~a.tin;
  c = 0;
  for (int p = 0; p < r; ++p)
    if (!((a.tin >> p) & 1u)) a.rest_out[c++] = out_of[p];
  a.n_rest = int64_t(1) << (r - a.t);
  const int64_t units = batch * a.n_rest;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(units, (int64_t)n_cus() * 8));
  permute_kernel<<<grid, kPermBlock, 0, (hipStream_t)stream>>>(a);
  QBE_HIP(hipGetLastError());
  return QBE_OK;
}

}  // namespace qbe
