// Fragment labelling on the device: connected components of the cells whose
// solid volume fraction exceeds a cut (Sections 4.2 and 4.3 delineate
// fragments at the volume-fraction contour), face connectivity, each
// component labelled with its smallest linear cell index (x fastest).
//
// Union-find on an int32 parent array that is the caller's label buffer:
// every parent index is at most its child's, and a root is only ever linked
// under a smaller root (atomicMin), so each tree's root is the minimum index
// of its component and the result does not depend on the order in which
// threads run.  Fragment ids follow label order through a two-level scan,
// and fragment masses go to exact 32-bit-chunk integer bins, so every output
// is deterministic and bit-exact.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fvk {

struct CclGrid {
  int nx, ny, nz;
  int64_t ncell;
};

__device__ __forceinline__ int ccl_parent(const int* L, int i) {
  return __hip_atomic_load(L + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of i: parents strictly decrease along the chain, so this ends.
__device__ __forceinline__ int ccl_find(const int* L, int i) {
  int p = ccl_parent(L, i);
  while (p != i) {
    i = p;
    p = ccl_parent(L, i);
  }
  return i;
}

// Join the trees of a and b.  Each retry continues from a strictly smaller
// index (the parent that displaced b), so the loop ends.
__device__ void ccl_unite(int* L, int a, int b) {
  while (true) {
    a = ccl_find(L, a);
    b = ccl_find(L, b);
    if (a == b) return;
    if (a > b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(L + b, a);
    if (old == b) return;  // b was a root and now hangs under a
    b = old;               // b had been linked to old < b: join a with old
  }
}

template <class T>
__global__ void __launch_bounds__(256) ccl_init_kernel(const T* phi_s, double cut, CclGrid g,
                                                       int* L) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  L[c] = (double)phi_s[c] > cut ? (int)c : -1;
}

__global__ void __launch_bounds__(256) ccl_merge_kernel(CclGrid g, int* L) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  if (ccl_parent(L, (int)c) < 0) return;
  const int x = (int)(c % g.nx);
  const int64_t r = c / g.nx;
  const int y = (int)(r % g.ny);
  const int z = (int)(r / g.ny);
  // material cells never change sign, so the test on a neighbour is stable
  if (x > 0 && ccl_parent(L, (int)c - 1) >= 0) ccl_unite(L, (int)c, (int)c - 1);
  if (y > 0 && ccl_parent(L, (int)(c - g.nx)) >= 0) ccl_unite(L, (int)c, (int)(c - g.nx));
  const int64_t pl = (int64_t)g.nx * g.ny;
  if (z > 0 && ccl_parent(L, (int)(c - pl)) >= 0) ccl_unite(L, (int)c, (int)(c - pl));
}

__global__ void __launch_bounds__(256) ccl_compress_kernel(CclGrid g, int* L) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int p = L[c];
  if (p < 0 || p == (int)c) return;
  L[c] = ccl_find(L, p);
}

// number of roots (L[c] == c) before this thread in its block, and the block
// total, through wave ballots
__device__ __forceinline__ int ccl_block_rank(bool root, int* sh, int& total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long m = __ballot(root);
  const int below = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) sh[wid] = __popcll(m);
  __syncthreads();
  int before = 0;
  total = 0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nw; ++w) {
    if (w < wid) before += sh[w];
    total += sh[w];
  }
  return before + below;
}

__global__ void __launch_bounds__(256) ccl_count_kernel(CclGrid g, const int* L, int* bcount) {
  __shared__ int sh[4];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool root = c < g.ncell && L[c] == (int)c;
  int total;
  ccl_block_rank(root, sh, total);
  if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// Exclusive scan of the per-block root counts in one block of 1024 threads;
// the grand total goes to *n_root.
__global__ void __launch_bounds__(1024) ccl_scan_kernel(int nblk, int* bcount, long long* n_root) {
  __shared__ long long sh[1024];
  long long carry = 0;
  for (int base = 0; base < nblk; base += 1024) {
    const int i = base + (int)threadIdx.x;
    const long long v = i < nblk ? bcount[i] : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const long long add = threadIdx.x >= (unsigned)o ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nblk) bcount[i] = (int)(carry + sh[threadIdx.x] - v);
    const long long tot = sh[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) *n_root = carry;
}

// Fragment id of every root in label order, and the label of every fragment.
__global__ void __launch_bounds__(256) ccl_assign_kernel(CclGrid g, const int* L, const int* boff,
                                                         int* fid, int* flabel) {
  __shared__ int sh[4];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool root = c < g.ncell && L[c] == (int)c;
  int total;
  const int rank = ccl_block_rank(root, sh, total);
  if (root) {
    const int f = boff[blockIdx.x] + rank;
    fid[c] = f;
    flabel[f] = (int)c;
  }
}

// Per-fragment exact mass bins, cell counts and boundary flags.
template <class T>
__global__ void __launch_bounds__(256) ccl_stats_kernel(CclGrid g, const int* L, const int* fid,
                                                        const T* mass_s,
                                                        unsigned long long* fbins,
                                                        unsigned long long* fcount,
                                                        unsigned int* fflag) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.ncell) return;
  const int r = L[c];
  if (r < 0) return;
  const int f = fid[r];
  bin_add(fbins + (size_t)f * NBINS, (double)mass_s[c]);
  atomicAdd(fcount + f, 1ull);
  const int x = (int)(c % g.nx);
  const int64_t q = c / g.nx;
  const int y = (int)(q % g.ny);
  const int z = (int)(q / g.ny);
  const bool edge = (g.nx > 1 && (x == 0 || x == g.nx - 1)) ||
                    (g.ny > 1 && (y == 0 || y == g.ny - 1)) ||
                    (g.nz > 1 && (z == 0 || z == g.nz - 1));
  if (edge) atomicOr(fflag + f, 1u);
}

}  // namespace fvk
