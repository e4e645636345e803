// Topology of a T4 mesh, built once per mesh on the device:
//   1. faces (Sec. 3.2, Alg. 1): the 4T face keys are bucketed by their
//      smallest node and sorted inside the bucket; equal keys pair up into
//      interior faces (two tets), singletons are exterior faces; a key seen
//      more than twice is a non-manifold mesh;
//   2. node -> face incidence: for each node the faces whose smoothing-domain
//      support (the face's 3 nodes plus the opposite vertex of each tet)
//      contains it;
//   3. the 3x3-block CSR pattern: node J is a neighbour of node I when some
//      face's support holds both -- exactly the positions of Eq. 12's
//      triplets;
//   4. assembly tiles: runs of consecutive node rows whose blocks fit in LDS.
#include "ctx.h"

namespace sfem {

namespace {

__device__ __forceinline__ void sort3(int& a, int& b, int& c) {
  int t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

// Face of tet t opposite its local vertex lf: bucket = smallest node, value
// encodes (middle, largest) node and the (tet, local face) payload.
// Largest vertex-id spread (max - min) of a tet: per-block maxima.
__global__ void k_tet_spread(const int32_t* __restrict__ tets, int64_t T,
                             int32_t* __restrict__ part) {
  int m = 0;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < T;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int4 v = reinterpret_cast<const int4*>(tets)[t];
    const int lo = min(min(v.x, v.y), min(v.z, v.w)), hi = max(max(v.x, v.y), max(v.z, v.w));
    m = max(m, hi - lo);
  }
  m = wave_max(m);
  __shared__ int sm[4];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = max(max(sm[0], sm[1]), max(sm[2], sm[3]));
}

// Face entries bucketed by their smallest vertex a; the value packs the
// other two vertices relative to a (b - a, c - a < W, W = largest tet
// vertex-id spread + 1) above the entry index 4t + lf.
__global__ void k_face_entries(const int32_t* __restrict__ tets, int64_t T, uint64_t W,
                               int32_t* __restrict__ bucket, uint64_t* __restrict__ vals) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int4 v4 = reinterpret_cast<const int4*>(tets)[t];
  int v[4] = {v4.x, v4.y, v4.z, v4.w};
  const uint64_t T4 = uint64_t(4) * uint64_t(T);
#pragma unroll
  for (int lf = 0; lf < 4; ++lf) {
    int a = v[(lf + 1) & 3], b = v[(lf + 2) & 3], c = v[(lf + 3) & 3];
    sort3(a, b, c);
    bucket[4 * t + lf] = a;
    vals[4 * t + lf] =
        (uint64_t(b - a) * W + uint64_t(c - a)) * T4 + uint64_t(4 * t + lf);
  }
}

// Per smallest node: count distinct keys; flag runs longer than 2.
__global__ void k_face_count(const int32_t* __restrict__ ptr, const uint64_t* __restrict__ v,
                             int64_t N, uint64_t T4, int32_t* __restrict__ cnt,
                             int32_t* __restrict__ err) {
  int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int b = ptr[a], e = ptr[a + 1];
  int n = 0, run = 0;
  uint64_t prev = ~uint64_t(0);
  for (int i = b; i < e; ++i) {
    uint64_t key = v[i] / T4;
    if (key != prev) {
      ++n;
      run = 1;
      prev = key;
    } else if (++run > 2) {
      atomicOr(err, 1);
    }
  }
  cnt[a] = n;
}

__global__ void k_face_write(const int32_t* __restrict__ ptr, const uint64_t* __restrict__ v,
                             const int32_t* __restrict__ fptr, const int32_t* __restrict__ tets,
                             int64_t N, uint64_t W, uint64_t T4, int32_t* __restrict__ face,
                             unsigned long long* __restrict__ n_ext) {
  int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= N) return;
  int b = ptr[a], e = ptr[a + 1];
  int f = fptr[a];
  unsigned long long ext = 0;
  for (int i = b; i < e;) {
    uint64_t key = v[i] / T4;
    uint64_t pay1 = v[i] % T4;
    int t1 = int(pay1 >> 2), o1 = tets[pay1];
    int t2 = -1, o2 = -1;
    int step = 1;
    if (i + 1 < e && v[i + 1] / T4 == key) {
      uint64_t pay2 = v[i + 1] % T4;
      t2 = int(pay2 >> 2);
      o2 = tets[pay2];
      step = 2;
    } else {
      ++ext;
    }
    int* row = face + int64_t(f) * kFaceStride;
    row[0] = int(a);
    row[1] = int(a + int64_t(key / W));
    row[2] = int(a + int64_t(key % W));
    row[3] = o1;
    row[4] = o2;
    row[5] = t1;
    row[6] = t2;
    row[7] = 0;
    ++f;
    i += step;
  }
  if (ext) atomicAdd(n_ext, ext);
}

// Incidence entries: 5 per face (support nodes); the 5th of an exterior face
// goes to the spare bucket N.
__global__ void k_inc_entries(const int32_t* __restrict__ face, int64_t nf, int64_t N,
                              int32_t* __restrict__ bucket, uint32_t* __restrict__ vals) {
  int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int* row = face + f * kFaceStride;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    int n = row[s];
    bucket[5 * f + s] = n >= 0 ? n : int(N);
    vals[5 * f + s] = uint32_t(f);
  }
}

// Block pattern of node rows, one wave per node: candidate neighbours are the
// support nodes of the node's incident smoothing domains (rows of STRIDE
// ints, the first PER of them support nodes or -1); duplicates are dropped.
// Pass 0 counts distinct neighbours, pass 1 writes them in ascending order.
// Candidate lists up to kPatLds are staged in LDS with duplicates marked -1;
// longer ones (far beyond any T4 mesh of sane quality) are read from HBM.
constexpr int kPatWaves = 4;
constexpr int kPatLds = 1024;  // <= 16 candidates per lane

template <int PASS, int STRIDE, int PER>
__global__ void __launch_bounds__(kPatWaves * kWave)
    k_pattern(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
              const int32_t* __restrict__ rows, int64_t N, int32_t* __restrict__ deg,
              const int32_t* __restrict__ bptr, int32_t* __restrict__ bcol) {
  __shared__ int32_t cand[kPatWaves][kPatLds];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int64_t I = int64_t(blockIdx.x) * kPatWaves + wid;
  int b = 0, m = 0;
  if (I < N) {
    b = inc_ptr[I];
    m = PER * (inc_ptr[I + 1] - b);
  }
  const bool staged = m <= kPatLds;
  int32_t* s = cand[wid];
  // candidate i: support node i % PER of the (i / PER)-th incident domain
  auto cand_at = [&](int i) -> int32_t {
    return rows[int64_t(inc[b + i / PER]) * STRIDE + i % PER];
  };
  if (staged)
    for (int i = lane; i < m; i += kWave) s[i] = cand_at(i);
  __syncthreads();
  unsigned dup = 0;
  if (staged) {
    int k = 0;
    for (int i = lane; i < m; i += kWave, ++k) {
      int32_t v = s[i];
      bool d = v < 0;
      for (int j = 0; j < i && !d; ++j) d = (s[j] == v);
      if (d) dup |= 1u << k;
    }
  }
  __syncthreads();
  if (staged) {
    int k = 0;
    for (int i = lane; i < m; i += kWave, ++k)
      if ((dup >> k) & 1u) s[i] = -1;
  }
  __syncthreads();
  if (I >= N) return;
  int cnt = 0;
  if (staged) {
    for (int i = lane; i < m; i += kWave) {
      int32_t v = s[i];
      if (v < 0) continue;
      if (PASS == 0) {
        ++cnt;
      } else {
        int r = 0;
        for (int j = 0; j < m; ++j) {
          int32_t w = s[j];
          r += (w >= 0 && w < v);
        }
        bcol[bptr[I] + r] = v;
      }
    }
  } else {
    auto first = [&](int i, int32_t v) {
      for (int j = 0; j < i; ++j)
        if (cand_at(j) == v) return false;
      return true;
    };
    for (int i = lane; i < m; i += kWave) {
      int32_t v = cand_at(i);
      if (v < 0 || !first(i, v)) continue;
      if (PASS == 0) {
        ++cnt;
      } else {
        int r = 0;
        for (int j = 0; j < m; ++j) {
          int32_t w = cand_at(j);
          if (w >= 0 && w < v && first(j, w)) ++r;
        }
        bcol[bptr[I] + r] = v;
      }
    }
  }
  if (PASS == 0) {
    cnt = wave_sum(cnt);
    if (lane == 0) deg[I] = cnt;
  }
}

// out[0] = largest node degree; out[1] = 1 if some node is in no tet;
// out[2] = most incident faces of one node.
__global__ void k_maxdeg(const int32_t* __restrict__ bptr, const int32_t* __restrict__ inc_ptr,
                         int64_t N, int* __restrict__ out) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  int d = bptr[I + 1] - bptr[I];
  atomicMax(out, d);
  atomicMax(out + 2, inc_ptr[I + 1] - inc_ptr[I]);
  if (d == 0) atomicOr(out + 1, 1);
}

// Node I opens a new tile when floor(bptr[I] / C) differs from its
// predecessor's; C = capacity - maxdeg keeps every tile within capacity.
__global__ void k_tiles(const int32_t* __restrict__ bptr, int64_t N, int C,
                        int32_t* __restrict__ tile_first, int n_tiles) {
  int64_t I = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (I >= N) return;
  int t = bptr[I] / C;
  if (I == 0 || bptr[I - 1] / C != t) tile_first[t] = int(I);
  if (I == N - 1) tile_first[n_tiles] = int(N);
}

// Per incidence entry of row I: I's index within its assembly tile (a
// tile holds at most kTileBlocks rows).  One wave per row.
__global__ void k_inc_rows(int64_t N, const int32_t* __restrict__ inc_ptr,
                           const int32_t* __restrict__ tile_first, int n_tiles,
                           uint16_t* __restrict__ irow) {
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x & (kWave - 1);
  if (I >= N) return;
  int lo = 0, hi = n_tiles - 1;  // the last tile t with tile_first[t] <= I
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tile_first[mid] <= int(I)) lo = mid;
    else hi = mid - 1;
  }
  const uint16_t li = uint16_t(int(I) - tile_first[lo]);
  for (int e = inc_ptr[I] + lane; e < inc_ptr[I + 1]; e += kWave) irow[e] = li;
}

// Slot map: for incidence entry e = (row node I, face f), the positions of
// f's support nodes among row I's block columns, 6 bits each (slot q in
// bits 6q..6q+5).  One wave per node row.
__global__ void k_slot_map(const int32_t* __restrict__ inc_ptr, const int32_t* __restrict__ inc,
                           const int32_t* __restrict__ face, const int32_t* __restrict__ bptr,
                           const int32_t* __restrict__ bcol, int64_t N,
                           uint32_t* __restrict__ slots) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t I = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  if (I >= N) return;
  const int rb = bptr[I], deg = bptr[I + 1] - rb;
  const int32_t* cols = bcol + rb;
  for (int e = inc_ptr[I] + lane; e < inc_ptr[I + 1]; e += kWave) {
    const int32_t* row = face + int64_t(inc[e]) * kFaceStride;
    uint32_t code = 0;
    for (int q = 0; q < 5; ++q) {
      const int J = row[q];
      if (J < 0) continue;
      int lo = 0, hi = deg - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cols[mid] < J) lo = mid + 1;
        else hi = mid;
      }
      code |= uint32_t(lo) << (6 * q);
    }
    slots[e] = code;
  }
}

// Degenerate tet check: |det| must exceed a tiny fraction of the product of
// its edge lengths from vertex 0.
__global__ void k_check_tets(const double* __restrict__ xyz, const int32_t* __restrict__ tets,
                             int64_t T, int32_t* __restrict__ err) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= T) return;
  int4 v = reinterpret_cast<const int4*>(tets)[t];
  const double* p0 = xyz + 3 * int64_t(v.x);
  const double* p1 = xyz + 3 * int64_t(v.y);
  const double* p2 = xyz + 3 * int64_t(v.z);
  const double* p3 = xyz + 3 * int64_t(v.w);
  double e1[3], e2[3], e3[3];
  for (int i = 0; i < 3; ++i) {
    e1[i] = p1[i] - p0[i];
    e2[i] = p2[i] - p0[i];
    e3[i] = p3[i] - p0[i];
  }
  double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
               e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
  double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
  double l3 = sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
  if (!(fabs(det) > 1e-12 * l1 * l2 * l3)) atomicOr(err, 2);
}

template <typename T>
T read_scalar(const T* dev, hipStream_t s) {
  T h;
  SFEM_HIP(hipMemcpyAsync(&h, dev, sizeof(T), hipMemcpyDeviceToHost, s));
  SFEM_HIP(hipStreamSynchronize(s));
  return h;
}

}  // namespace

// Block pattern (bptr, bcol, nb, maxdeg) of the smoothing domains given by
// a node -> domain incidence and the domains' support rows, then the
// assembly tiles.  Returns the most domains holding one node.
template <int STRIDE, int PER>
int build_pattern(Ctx& c, const int32_t* inc_ptr, const int32_t* inc, const int32_t* rows) {
  hipStream_t s = c.stream;
  Topology& tp = c.topo;
  const int64_t N = c.N;
  const int B = 256;
  TmpBuf<int32_t> deg(N + 1, s);
  tp.bptr.reserve(N + 1);
  const int pg = div_up(N, kPatWaves);
  k_pattern<0, STRIDE, PER><<<pg, kPatWaves * kWave, 0, s>>>(inc_ptr, inc, rows, N, deg.get(),
                                                               nullptr, nullptr);
  SFEM_HIP(hipGetLastError());
  exclusive_scan_i32(deg.get(), tp.bptr.get(), N, s);
  tp.nb = read_scalar(tp.bptr.get() + N, s);
  SFEM_REQUIRE(tp.nb >= N, SFEM_EMESH, "a node belongs to no tetrahedron");
  SFEM_REQUIRE(9 * tp.nb < (int64_t(1) << 31), SFEM_EINVAL,
               "matrix too large for int32 CSR indices");
  tp.bcol.reserve(tp.nb);
  k_pattern<1, STRIDE, PER><<<pg, kPatWaves * kWave, 0, s>>>(inc_ptr, inc, rows, N, nullptr,
                                                               tp.bptr.get(), tp.bcol.get());
  SFEM_HIP(hipGetLastError());
  deg.release();

  TmpBuf<int> md(3, s);
  SFEM_HIP(hipMemsetAsync(md.get(), 0, 3 * sizeof(int), s));
  k_maxdeg<<<div_up(N, B), B, 0, s>>>(tp.bptr.get(), inc_ptr, N, md.get());
  SFEM_HIP(hipGetLastError());
  tp.maxdeg = read_scalar(md.get(), s);
  const int isolated = read_scalar(md.get() + 1, s);
  const int max_inc = read_scalar(md.get() + 2, s);
  md.release();
  SFEM_REQUIRE(!isolated, SFEM_EMESH, "a node belongs to no tetrahedron");
  SFEM_REQUIRE(tp.maxdeg <= kMaxDeg && 2 * tp.maxdeg < kTileBlocks, SFEM_EMESH,
               "a node has more than 64 neighbours (" + std::to_string(tp.maxdeg) + ")");
  SFEM_REQUIRE(max_inc < 4096, SFEM_EMESH,
               "a node lies in more than 4095 smoothing domains (" + std::to_string(max_inc) +
                   ")");

  const int C = kTileBlocks - tp.maxdeg;
  const int last = read_scalar(tp.bptr.get() + (N - 1), s);
  tp.n_tiles = last / C + 1;
  tp.tile_first.reserve(tp.n_tiles + 1);
  k_tiles<<<div_up(N, B), B, 0, s>>>(tp.bptr.get(), N, C, tp.tile_first.get(), tp.n_tiles);
  SFEM_HIP(hipGetLastError());
  return max_inc;
}

template int build_pattern<kEdgeSup, kEdgeSup>(Ctx&, const int32_t*, const int32_t*,
                                              const int32_t*);

void build_topology(Ctx& c) {
  hipStream_t s = c.stream;
  Topology& tp = c.topo;
  tp.valid = false;
  const int64_t N = c.N, T = c.T;
  tp.N = N;
  tp.T = T;
  const int B = 256;

  TmpBuf<int32_t> err(1, s);
  SFEM_HIP(hipMemsetAsync(err.get(), 0, sizeof(int32_t), s));
  k_check_tets<<<div_up(T, B), B, 0, s>>>(c.xyz.get(), c.tets.get(), T, err.get());
  SFEM_HIP(hipGetLastError());

  // 1. faces
  const int64_t n4 = 4 * T;
  TmpBuf<int32_t> fb(n4, s), fptr(N + 1, s), fcnt(N + 1, s);
  TmpBuf<uint64_t> fv(n4, s), fs(n4, s);
  // key base: the largest vertex-id spread of a tet (small for banded
  // numberings; a batch of meshes never has a tet spanning two meshes)
  {
    const int G = int(std::min<int64_t>(1024, div_up(T, B)));
    TmpBuf<int32_t> part(G, s);
    k_tet_spread<<<G, B, 0, s>>>(c.tets.get(), T, part.get());
    SFEM_HIP(hipGetLastError());
    std::vector<int32_t> hp(G);
    SFEM_HIP(hipMemcpyAsync(hp.data(), part.get(), sizeof(int32_t) * G, hipMemcpyDeviceToHost,
                            s));
    SFEM_HIP(hipStreamSynchronize(s));
    tp.key_w = 1 + *std::max_element(hp.begin(), hp.end());
  }
  const uint64_t W = uint64_t(tp.key_w);
  if (double(W) * double(W) * 4.0 * double(T) >= 9.2e18)
    throw Error{SFEM_EINVAL, "face keys overflow: (largest tet vertex-id spread + 1)^2 * 4 n_tets "
                             "must be < 2^63 (renumber the nodes)"};
  k_face_entries<<<div_up(T, B), B, 0, s>>>(c.tets.get(), T, W, fb.get(), fv.get());
  SFEM_HIP(hipGetLastError());
  bucket_sort_u64(fb.get(), fv.get(), n4, int(N), fptr.get(), fs.get(), s);
  k_face_count<<<div_up(N, B), B, 0, s>>>(fptr.get(), fs.get(), N, uint64_t(n4), fcnt.get(),
                                          err.get());
  SFEM_HIP(hipGetLastError());
  TmpBuf<int32_t> face_ofs(N + 1, s);
  exclusive_scan_i32(fcnt.get(), face_ofs.get(), N, s);
  const int32_t h_err = read_scalar(err.get(), s);
  if (h_err)
    throw Error{SFEM_EMESH, (h_err & 2) ? "degenerate (zero-volume) tetrahedron in mesh"
                                        : "non-manifold mesh: a face is shared by more than two tets"};
  tp.nf = read_scalar(face_ofs.get() + N, s);
  SFEM_REQUIRE(tp.nf >= 4, SFEM_EHIP, "face extraction produced no faces");
  tp.face.reserve(size_t(tp.nf) * kFaceStride);
  TmpBuf<unsigned long long> next(1, s);
  SFEM_HIP(hipMemsetAsync(next.get(), 0, sizeof(unsigned long long), s));
  k_face_write<<<div_up(N, B), B, 0, s>>>(fptr.get(), fs.get(), face_ofs.get(), c.tets.get(), N,
                                          W, uint64_t(n4), tp.face.get(), next.get());
  SFEM_HIP(hipGetLastError());
  tp.ne = int64_t(read_scalar(next.get(), s));
  // the face sort's buffers go before the incidence is built
  fb.release();
  fv.release();
  fs.release();
  fptr.release();
  fcnt.release();
  face_ofs.release();
  next.release();

  // 2. node -> face incidence
  const int64_t n5 = 5 * tp.nf;
  TmpBuf<int32_t> ib(n5, s);
  TmpBuf<uint32_t> iv(n5, s);
  k_inc_entries<<<div_up(tp.nf, B), B, 0, s>>>(tp.face.get(), tp.nf, N, ib.get(), iv.get());
  SFEM_HIP(hipGetLastError());
  tp.inc_ptr.reserve(N + 2);
  tp.inc.reserve(n5);
  // the spare bucket N only collects padding and is never read: left unsorted
  bucket_sort_u32(ib.get(), iv.get(), n5, int(N + 1), tp.inc_ptr.get(),
                  reinterpret_cast<uint32_t*>(tp.inc.get()), s, int(N));
  ib.release();
  iv.release();
  tp.n_inc = read_scalar(tp.inc_ptr.get() + N, s);

  // 3.-4. block pattern of the face domains, assembly tiles
  tp.max_inc = build_pattern<kFaceStride, 5>(c, tp.inc_ptr.get(), tp.inc.get(), tp.face.get());
  tp.slot.reserve(tp.n_inc);
  k_slot_map<<<div_up(N * kWave, B), B, 0, s>>>(tp.inc_ptr.get(), tp.inc.get(), tp.face.get(),
                                                tp.bptr.get(), tp.bcol.get(), N, tp.slot.get());
  SFEM_HIP(hipGetLastError());
  tp.irow.reserve(tp.n_inc);
  k_inc_rows<<<div_up(N * kWave, B), B, 0, s>>>(N, tp.inc_ptr.get(), tp.tile_first.get(),
                                                tp.n_tiles, tp.irow.get());
  SFEM_HIP(hipGetLastError());
  face_bounds(c);
  err.release();
  SFEM_HIP(hipStreamSynchronize(s));
  if (c.domain == SFEM_DOMAIN_EDGE) build_edge_topology(c);
  tp.valid = true;
}

}  // namespace sfem
