// Reverse Cuthill-McKee numbering of a tet mesh's nodes, on the device.
//
// Unstructured generators (the TetGen files the paper reads, Sec. 3.2)
// number nodes arbitrarily; the path wants neighbouring nodes close in
// number (small face-key base, local x-gathers in the row kernels).  The
// ordering is the classic one, made level-synchronous:
//   graph       nodes adjacent when they share a tet (the tets' edges);
//   start       George & Liu (1979): r = least (deg, id) node still to be
//               numbered; while the least-(deg, id) node x of r's last BFS
//               level has a deeper level structure, r = x;
//   numbering   Cuthill & McKee (1969): breadth-first from r, every node
//               numbering its unnumbered neighbours by increasing (deg, id).
//               Level L+1 is therefore ordered by (number of the earliest-
//               numbered neighbour in level L, deg, id): one device BFS
//               step marks the level and takes that minimum with atomicMin,
//               a bucket sort by the minimum (then (deg, id) inside each
//               bucket) gives the level's order;
//   components  one after the other, each from its own start;
//   reverse     George (1971): perm[new] = CM order[N - 1 - new].
// The result is a deterministic function of the mesh (no dependence on the
// order in which the device threads run).
#include "ctx.h"

namespace sfem {

namespace {

constexpr int kB = 256;

// 12 directed edges per tet, bucketed by source: value (target << 32 | tet)
// is distinct within a bucket.
__global__ void k_edge_entries(const int32_t* __restrict__ tets, int64_t T,
                               int32_t* __restrict__ bucket, uint64_t* __restrict__ vals) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 12 * T) return;
  const int64_t t = i / 12;
  const int k = int(i % 12), a = k / 3, j = k % 3, b = j < a ? j : j + 1;
  bucket[i] = tets[4 * t + a];
  vals[i] = (uint64_t(uint32_t(tets[4 * t + b])) << 32) | uint32_t(t);
}

// Distinct targets of each node's sorted entries: count, then write.
__global__ void k_unique(int64_t N, const int32_t* __restrict__ eptr,
                         const uint64_t* __restrict__ ev, const int32_t* __restrict__ aptr,
                         int32_t* __restrict__ deg, int32_t* __restrict__ adj) {
  const int64_t v = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= N) return;
  int n = 0, o = adj ? aptr[v] : 0;
  uint32_t prev = 0xffffffffu;
  for (int k = eptr[v]; k < eptr[v + 1]; ++k) {
    const uint32_t w = uint32_t(ev[k] >> 32);
    if (w != prev) {
      if (adj) adj[o + n] = int32_t(w);
      ++n;
      prev = w;
    }
  }
  if (deg) deg[v] = n;
}

__global__ void k_fill_i32(int64_t n, int32_t* __restrict__ a, int32_t v) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// lev = -1 for nodes still to be numbered (pos < 0), -2 otherwise.
__global__ void k_bfs_reset(int64_t N, const int32_t* __restrict__ pos, int32_t* __restrict__ lev) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) lev[i] = pos[i] < 0 ? -1 : -2;
}

// Least (deg << 32 | id) over the nodes still to be numbered.
__global__ void k_argmin_free(int64_t N, const int32_t* __restrict__ pos,
                              const int32_t* __restrict__ deg,
                              unsigned long long* __restrict__ best) {
  __shared__ unsigned long long s[kB / kWave];
  unsigned long long m = ~0ull;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N;
       i += int64_t(gridDim.x) * blockDim.x)
    if (pos[i] < 0) {
      const unsigned long long k = (uint64_t(uint32_t(deg[i])) << 32) | uint32_t(i);
      m = k < m ? k : m;
    }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(m, o);
    m = w < m ? w : m;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kB / kWave; ++w) m = s[w] < m ? s[w] : m;
    atomicMin(best, m);
  }
}

// Least (deg << 32 | id) over a list of nodes.
__global__ void k_argmin_list(const int32_t* __restrict__ list, int n,
                              const int32_t* __restrict__ deg,
                              unsigned long long* __restrict__ best) {
  __shared__ unsigned long long s[kB / kWave];
  unsigned long long m = ~0ull;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int v = list[i];
    const unsigned long long k = (uint64_t(uint32_t(deg[v])) << 32) | uint32_t(v);
    m = k < m ? k : m;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(m, o);
    m = w < m ? w : m;
  }
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kB / kWave; ++w) m = s[w] < m ? s[w] : m;
    atomicMin(best, m);
  }
}

// One BFS step: every unvisited (lev == -1) neighbour of the frontier gets
// level L+1 and is appended to `next`.  With pos given (numbering pass),
// minpos[v] takes the least number of v's neighbours in the frontier.
__global__ void k_bfs_step(const int32_t* __restrict__ front, int nf,
                           const int32_t* __restrict__ aptr, const int32_t* __restrict__ adj,
                           int32_t* __restrict__ lev, int L, const int32_t* __restrict__ pos,
                           int32_t* __restrict__ minpos, int32_t* __restrict__ next,
                           int32_t* __restrict__ cnt) {
  // one wave per frontier node, lanes over its neighbours
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t w = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (w >= nf) return;
  const int u = front[w];
  const int pu = pos ? pos[u] : 0;
  for (int k = aptr[u] + lane; k < aptr[u + 1]; k += kWave) {
    const int v = adj[k];
    const int old = atomicCAS(&lev[v], -1, L + 1);
    if (old == -1) next[atomicAdd(cnt, 1)] = v;
    if (pos && (old == -1 || old == L + 1)) atomicMin(&minpos[v], pu);
  }
}

// Sort keys of a new level: bucket = minpos - (first number of the previous
// level), value = deg << 32 | id.
__global__ void k_level_keys(const int32_t* __restrict__ next, int m,
                             const int32_t* __restrict__ minpos, const int32_t* __restrict__ deg,
                             int first, int32_t* __restrict__ bucket,
                             uint64_t* __restrict__ vals) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int v = next[i];
  bucket[i] = minpos[v] - first;
  vals[i] = (uint64_t(uint32_t(deg[v])) << 32) | uint32_t(v);
}

// Numbers of the sorted level: pos[v] = first + i, order[first + i] = v.
__global__ void k_level_assign(const uint64_t* __restrict__ sorted, int m, int first,
                               int32_t* __restrict__ pos, int32_t* __restrict__ order,
                               int32_t* __restrict__ front) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int v = int(uint32_t(sorted[i]));
  pos[v] = first + i;
  order[first + i] = v;
  front[i] = v;
}

__global__ void k_set_start(int v, int p, int32_t* __restrict__ pos, int32_t* __restrict__ order,
                            int32_t* __restrict__ lev, int32_t* __restrict__ front) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    if (pos) pos[v] = p;
    if (order) order[p] = v;
    lev[v] = 0;
    front[0] = v;
  }
}

__global__ void k_reverse(int64_t N, const int32_t* __restrict__ order, int32_t* __restrict__ perm) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) perm[i] = order[N - 1 - i];
}

__global__ void k_inverse(int64_t N, const int32_t* __restrict__ perm, int32_t* __restrict__ inv) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < N) inv[perm[i]] = int32_t(i);
}

__global__ void k_gather_xyz(int64_t N, const int32_t* __restrict__ perm,
                             const double* __restrict__ xyz, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t o = perm[i];
  out[3 * i + 0] = xyz[3 * o + 0];
  out[3 * i + 1] = xyz[3 * o + 1];
  out[3 * i + 2] = xyz[3 * o + 2];
}

__global__ void k_map_tets(int64_t n, const int32_t* __restrict__ inv,
                           const int32_t* __restrict__ tets, int32_t* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = inv[tets[i]];
}

__global__ void k_perm_hits(int64_t N, const int32_t* __restrict__ perm,
                            int32_t* __restrict__ hits, int32_t* __restrict__ err) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int32_t v = perm[i];
  if (v < 0 || v >= N) atomicOr(err, 1);
  else if (atomicAdd(&hits[v], 1) != 0) atomicOr(err, 1);
}

template <typename T>
T read1(const T* d, hipStream_t s) {
  T h;
  SFEM_HIP(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  return h;
}

struct NodeGraph {
  DBuf<int32_t> aptr, adj, deg;
};

void node_graph(hipStream_t s, int64_t N, int64_t T, const int32_t* tets, NodeGraph& g) {
  const int64_t ne = 12 * T;
  DBuf<int32_t> bucket, eptr;
  DBuf<uint64_t> vals, sorted;
  bucket.reserve(ne);
  vals.reserve(ne);
  sorted.reserve(ne);
  eptr.reserve(N + 1);
  k_edge_entries<<<div_up(ne, kB), kB, 0, s>>>(tets, T, bucket.get(), vals.get());
  SFEM_HIP(hipGetLastError());
  bucket_sort_u64(bucket.get(), vals.get(), ne, int(N), eptr.get(), sorted.get(), s);
  g.deg.reserve(N);
  g.aptr.reserve(N + 1);
  k_unique<<<div_up(N, kB), kB, 0, s>>>(N, eptr.get(), sorted.get(), nullptr, g.deg.get(), nullptr);
  SFEM_HIP(hipGetLastError());
  exclusive_scan_i32(g.deg.get(), g.aptr.get(), N, s);
  const int32_t na = read1(g.aptr.get() + N, s);
  g.adj.reserve(na > 0 ? na : 1);
  k_unique<<<div_up(N, kB), kB, 0, s>>>(N, eptr.get(), sorted.get(), g.aptr.get(), nullptr,
                                        g.adj.get());
  SFEM_HIP(hipGetLastError());
  SFEM_HIP(hipStreamSynchronize(s));
}

// Depth of r's level structure over the nodes with lev == -1 after a reset,
// and the least-(deg, id) node of its last level.
int bfs_depth(hipStream_t s, int64_t N, const NodeGraph& g, int r, const int32_t* pos,
              int32_t* lev, int32_t* f0, int32_t* f1, int32_t* cnt, unsigned long long* best,
              int& last_best) {
  k_bfs_reset<<<div_up(N, kB), kB, 0, s>>>(N, pos, lev);
  k_set_start<<<1, 64, 0, s>>>(r, 0, nullptr, nullptr, lev, f0);
  SFEM_HIP(hipGetLastError());
  int nf = 1, L = 0;
  int32_t* front = f0;
  int32_t* next = f1;
  for (;;) {
    SFEM_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t), s));
    k_bfs_step<<<div_up(int64_t(nf) * kWave, kB), kB, 0, s>>>(front, nf, g.aptr.get(),
                                                             g.adj.get(), lev, L, nullptr,
                                                             nullptr, next, cnt);
    SFEM_HIP(hipGetLastError());
    const int m = read1(cnt, s);
    if (m == 0) break;
    std::swap(front, next);
    nf = m;
    ++L;
  }
  SFEM_HIP(hipMemsetAsync(best, 0xff, sizeof(unsigned long long), s));
  k_argmin_list<<<std::min(div_up(nf, kB), 1024), kB, 0, s>>>(front, nf, g.deg.get(), best);
  SFEM_HIP(hipGetLastError());
  last_best = int(uint32_t(read1(best, s)));
  return L + 1;
}

}  // namespace

void rcm_order(hipStream_t s, int64_t N, int64_t T, const int32_t* tets, int32_t* perm) {
  NodeGraph g;
  node_graph(s, N, T, tets, g);
  DBuf<int32_t> pos, order, lev, minpos, f0, f1, cnt, bucket, bptr;
  DBuf<uint64_t> vals, sorted;
  DBuf<unsigned long long> best;
  pos.reserve(N);
  order.reserve(N);
  lev.reserve(N);
  minpos.reserve(N);
  f0.reserve(N);
  f1.reserve(N);
  bucket.reserve(N);
  bptr.reserve(N + 1);
  vals.reserve(N);
  sorted.reserve(N);
  cnt.reserve(1);
  best.reserve(1);
  k_fill_i32<<<div_up(N, kB), kB, 0, s>>>(N, pos.get(), -1);
  k_fill_i32<<<div_up(N, kB), kB, 0, s>>>(N, minpos.get(), 0x7fffffff);
  SFEM_HIP(hipGetLastError());
  int64_t numbered = 0;
  while (numbered < N) {
    // component seed and its George-Liu start
    SFEM_HIP(hipMemsetAsync(best.get(), 0xff, sizeof(unsigned long long), s));
    k_argmin_free<<<std::min(div_up(N, kB), 1024), kB, 0, s>>>(N, pos.get(), g.deg.get(),
                                                              best.get());
    SFEM_HIP(hipGetLastError());
    int r = int(uint32_t(read1(best.get(), s)));
    int x = 0;
    int depth = bfs_depth(s, N, g, r, pos.get(), lev.get(), f0.get(), f1.get(), cnt.get(),
                          best.get(), x);
    for (;;) {
      int x2 = 0;
      const int dx = bfs_depth(s, N, g, x, pos.get(), lev.get(), f0.get(), f1.get(), cnt.get(),
                               best.get(), x2);
      if (dx <= depth) break;
      r = x;
      depth = dx;
      x = x2;
    }
    // Cuthill-McKee numbering of the component, level by level
    k_bfs_reset<<<div_up(N, kB), kB, 0, s>>>(N, pos.get(), lev.get());
    k_set_start<<<1, 64, 0, s>>>(r, int(numbered), pos.get(), order.get(), lev.get(), f0.get());
    SFEM_HIP(hipGetLastError());
    int first = int(numbered), nf = 1, L = 0;
    numbered += 1;
    for (;;) {
      SFEM_HIP(hipMemsetAsync(cnt.get(), 0, sizeof(int32_t), s));
      k_bfs_step<<<div_up(int64_t(nf) * kWave, kB), kB, 0, s>>>(
          f0.get(), nf, g.aptr.get(), g.adj.get(), lev.get(), L, pos.get(), minpos.get(),
          f1.get(), cnt.get());
      SFEM_HIP(hipGetLastError());
      const int m = read1(cnt.get(), s);
      if (m == 0) break;
      k_level_keys<<<div_up(m, kB), kB, 0, s>>>(f1.get(), m, minpos.get(), g.deg.get(), first,
                                               bucket.get(), vals.get());
      SFEM_HIP(hipGetLastError());
      bucket_sort_u64(bucket.get(), vals.get(), m, nf, bptr.get(), sorted.get(), s);
      k_level_assign<<<div_up(m, kB), kB, 0, s>>>(sorted.get(), m, int(numbered), pos.get(),
                                                 order.get(), f0.get());
      SFEM_HIP(hipGetLastError());
      first = int(numbered);
      numbered += m;
      nf = m;
      ++L;
    }
  }
  k_reverse<<<div_up(N, kB), kB, 0, s>>>(N, order.get(), perm);
  SFEM_HIP(hipGetLastError());
  SFEM_HIP(hipStreamSynchronize(s));
}

bool is_permutation(hipStream_t s, int64_t N, const int32_t* perm) {
  DBuf<int32_t> hits, err;
  hits.reserve(N);
  err.reserve(1);
  k_fill_i32<<<div_up(N, kB), kB, 0, s>>>(N, hits.get(), 0);
  k_fill_i32<<<1, 64, 0, s>>>(1, err.get(), 0);
  k_perm_hits<<<div_up(N, kB), kB, 0, s>>>(N, perm, hits.get(), err.get());
  SFEM_HIP(hipGetLastError());
  return read1(err.get(), s) == 0;
}

void permute_mesh(hipStream_t s, int64_t N, int64_t T, const int32_t* perm, const double* xyz,
                  const int32_t* tets, double* xyz_out, int32_t* tets_out) {
  DBuf<int32_t> inv;
  inv.reserve(N);
  k_inverse<<<div_up(N, kB), kB, 0, s>>>(N, perm, inv.get());
  if (xyz && xyz_out) k_gather_xyz<<<div_up(N, kB), kB, 0, s>>>(N, perm, xyz, xyz_out);
  if (tets && tets_out)
    k_map_tets<<<div_up(4 * T, kB), kB, 0, s>>>(4 * T, inv.get(), tets, tets_out);
  SFEM_HIP(hipGetLastError());
  SFEM_HIP(hipStreamSynchronize(s));
}

}  // namespace sfem
