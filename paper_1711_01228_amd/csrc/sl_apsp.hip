// Hop distances of all vertex pairs and the weight row sums, built once per
// graph: d_ij is the graph-theoretic distance (Sec. 2, eq. 1; Sec. 5.1),
// w_ij = d_ij^-2, and W_i = sum_j w_ij is the diagonal of L^W (Prop. 2.1).
//
// Breadth-first search from kBfsSources (8192) sources at once.  Word k of
// vertex v (index 128 v + k) holds one bit per source base + 64 k + b.  Level l takes
// the level l-1 frontier F and finds N_l(v) = (OR of F over v's neighbours)
// & ~(N_{l-1}(v) | N_{l-2}(v)), the sources that reach v first at level l (no
// visited set: see bfs_settle).  N_l is kept in level slot l mod kBfsSlots and
// is the next frontier.  Beside each slot, one 64-bit mask per vertex marks the
// 16-byte chunks of its row that are not zero; only those chunks are written,
// and every reader loads a chunk only where its bit is set (the frontier is
// sparse at the first and last levels of a sweep).
//   k_bfs_gather  one wave per run of at most 16 CSR entries (built with the
//                 plan), each lane reading 16 bytes of a neighbour's 1 KiB
//                 frontier row per entry, all 16 loads in flight (level 1
//                 forms the sources' bits instead).  A run holds whole rows of
//                 degree <= 16: the wave owns them and writes their N_l.  A
//                 row of 17 to 64 entries (or an isolated vertex) takes a wave
//                 of its own, 16 entries a pass; a longer row a 1024-thread
//                 workgroup, whose waves combine their ORs through LDS.
// Every kBfsSlots levels, k_bfs_store turns the slots of that batch of levels
// into distance bytes: it transposes a 64-row by 8-word block through LDS into
// four bit planes of the level offset and one plane of "found", and writes
// the 16-byte lane chunks of the tile layout, 1 KiB contiguous per wave.  The
// first batch writes the sweep's whole column range (0 where no level found
// the pair); later batches merge into what is there.
// Levels after one that found nothing return at once (flags[l] is set by
// level l's update, flags[0] stands for the sources), so the host queues a
// batch of levels and reads one flag per batch.
#include "sl_device.h"
#include "sl_internal.h"

#include <algorithm>

namespace sl {

namespace {

constexpr int kGatherLanes = 64;              // lanes per neighbour row (16 bytes each; a lane group)
constexpr int kBfsWords = 2 * kGatherLanes;   // 64-bit words per vertex
constexpr int kBfsSources = 64 * kBfsWords;   // sources per sweep
constexpr int kBfsSlots = 16;                 // level bitmaps kept between stores of d
constexpr int kGatherGroups = 64 / kGatherLanes;
constexpr int kGatherRun = 16;                // CSR entries per lane group
constexpr int kWaveEntries = kGatherGroups * kGatherRun;  // CSR entries a wave takes per pass
static_assert(kGatherRun <= kGatherLanes && kWaveEntries <= 64, "a group's entries sit in its own lanes");
constexpr int kStoreWords = 8;                // words per row in one store block
constexpr int kXcds = 8;                      // workgroup b runs on XCD b mod 8
constexpr int kStoreBlocksPerLine = 128 / (8 * kStoreWords);  // word blocks of one 128-byte line

inline unsigned blocks_for(size_t items) { return (unsigned)((items + 255) / 256); }

// The sources' own bits (level 0): lane wl's chunk of vertex u, u's bit in the
// chunk of lane (u - base) / 128.  No slot holds level 0.
__device__ __forceinline__ ulonglong2 source_chunk(int u, int wl, int base) {
  const int sb = u - base;
  if (sb < 0 || sb >= kBfsSources || sb / 128 != wl) return make_ulonglong2(0ull, 0ull);
  const uint64_t bit = 1ull << (sb & 63);
  return (sb & 64) ? make_ulonglong2(0ull, bit) : make_ulonglong2(bit, 0ull);
}

// Chunk wl (16 bytes) of row v of a level slot whose chunk masks are M: zero
// unless the chunk's bit is set (the other chunks are not written).
__device__ __forceinline__ ulonglong2 masked_chunk(const ulonglong2* __restrict__ S, const uint64_t* __restrict__ M,
                                                   int v, int wl) {
  if (((M[v] >> wl) & 1ull) == 0) return make_ulonglong2(0ull, 0ull);
  return S[(size_t)v * (kBfsWords / 2) + wl];
}

// N_l for the two words (one 16-byte chunk q of vertex v) a lane holds of a
// row: the OR a of the neighbours' level l-1 bits without v's own bits of levels
// l-1 and l-2.  On an undirected graph a neighbour's distance from a source
// differs from v's by at most one, so a source in a is at distance l-2, l-1 or
// l from v, and the last exactly when it is in neither of v's two previous
// levels: no visited set is kept.  The whole wave calls this for one v (its 64
// lanes are the row's 64 chunks): the chunks that are not zero are stored and
// their mask written.  `found` is set when N_l is not empty (the wave raises
// the level's flag once).
__device__ __forceinline__ void bfs_settle(const ulonglong2* __restrict__ F, const uint64_t* __restrict__ M1,
                                          const ulonglong2* __restrict__ P2, const uint64_t* __restrict__ M2,
                                          ulonglong2* __restrict__ slot, uint64_t* __restrict__ mout, int v, int wl,
                                          int level, int base, uint64_t a0, uint64_t a1, bool& found) {
  ulonglong2 nw = make_ulonglong2(0ull, 0ull);
  if (a0 | a1) {
    // v's bits of levels l-1 and l-2 (level 0: the sources)
    const ulonglong2 p1 = level == 1 ? source_chunk(v, wl, base) : masked_chunk(F, M1, v, wl);
    const ulonglong2 p2 = level == 1   ? make_ulonglong2(0ull, 0ull)
                          : level == 2 ? source_chunk(v, wl, base)
                                       : masked_chunk(P2, M2, v, wl);
    nw = make_ulonglong2(a0 & ~(p1.x | p2.x), a1 & ~(p1.y | p2.y));
  }
  const bool nz = (nw.x | nw.y) != 0ull;
  const uint64_t m = __ballot(nz);
  if (nz) {
    slot[(size_t)v * (kBfsWords / 2) + wl] = nw;
    found = true;
  }
  if (wl == 0) mout[v] = m;
}

// flags[level] = 1, stored by one lane of the wave where any lane found a new
// pair (the lowest such lane, which is active here).
__device__ __forceinline__ void raise_flag(bool found, int32_t* __restrict__ flags, int level) {
  const uint64_t any = __ballot(found);
  if (found && (threadIdx.x & 63) == (unsigned)__builtin_ctzll(any)) flags[level] = 1;
}

constexpr int kGatherThreads = 1024;           // threads per gather workgroup (16 waves)
constexpr int kGatherWaves = kGatherThreads / 64;
constexpr int kMidMax = 64;                     // rows up to this degree take one wave

// The OR into (a0, a1) of the frontier chunks (lane wl's 16 bytes) of N
// neighbours: entry j's neighbour u (-1 for none) and, from level 2 on, its
// chunk mask are held by lane l0 + j.  At level 1 the frontier is the sources
// themselves.  A chunk is loaded only where its mask bit is set, and all N
// loads are issued before the first is used: a lane whose bit is clear leaves
// its load register unwritten (not zeroed, which would make each load wait for
// the one before) and masks it out afterwards.
template <int N>
__device__ __forceinline__ void frontier_or(const ulonglong2* __restrict__ F, int uj, uint64_t mj, int l0, int wl,
                                            int level, int base, uint64_t (&c0)[N], uint64_t (&c1)[N]) {
  if (level == 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int u = __builtin_amdgcn_readlane(uj, l0 + j);
      const ulonglong2 c = u < 0 ? make_ulonglong2(0ull, 0ull) : source_chunk(u, wl, base);
      c0[j] = c.x;
      c1[j] = c.y;
    }
    return;
  }
  ulonglong2 f[N];
  bool on[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int u = __builtin_amdgcn_readlane(uj, l0 + j);
    const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(mj >> 32), l0 + j) << 32) |
                       (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)mj, l0 + j);
    on[j] = (u >= 0) & (((m >> wl) & 1ull) != 0ull);
    if (on[j]) f[j] = F[(size_t)u * (kBfsWords / 2) + wl];
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    c0[j] = on[j] ? f[j].x : 0ull;
    c1[j] = on[j] ? f[j].y : 0ull;
  }
}

// The chunk mask of frontier row u, for lanes that hold an entry (0 for none
// and at level 1, where the frontier is formed, not read).
__device__ __forceinline__ uint64_t entry_mask(const uint64_t* __restrict__ M, int u, int level) {
  return u >= 0 && level > 1 ? M[u] : 0ull;
}

// The OR of lane wl's chunk over entries e0 .. e0 + kWaveEntries - 1 of a row
// (CSR entries from b), the wave's lane groups each taking kGatherRun of them:
// lane l holds entry e0 + l.
__device__ __forceinline__ void row_chunk_or(const ulonglong2* __restrict__ F, const uint64_t* __restrict__ M,
                                             const int32_t* __restrict__ col_idx, int b, int deg, int e0, int lane,
                                             int grp, int wl, int level, int base, uint64_t& a0, uint64_t& a1) {
  const int uj = e0 + lane < deg ? col_idx[b + e0 + lane] : -1;
  const uint64_t mj = entry_mask(M, uj, level);
  uint64_t c0[kGatherRun], c1[kGatherRun];
  frontier_or(F, uj, mj, kGatherRun * grp, wl, level, base, c0, c1);
#pragma unroll
  for (int j = 0; j < kGatherRun; ++j) {
    a0 |= c0[j];
    a1 |= c1[j];
  }
}

// OR across the wave's lane groups (lanes wl of every group): each group then holds the total.
__device__ __forceinline__ void groups_or(uint64_t& a0, uint64_t& a1) {
#pragma unroll
  for (int m = kGatherLanes; m < 64; m <<= 1) {
    a0 |= __shfl_xor(a0, m, 64);
    a1 |= __shfl_xor(a1, m, 64);
  }
}

// Three kinds of workgroup, by index:
//   [0, nbig)                 one row of degree above kMidMax each: its 16 waves
//                             share the entries, 256 per pass, and combine
//                             their ORs through LDS; wave 0's first group settles
//   [nbig, nbig + mid blocks) one row of degree 17 .. kMidMax, or an isolated
//                             vertex, per wave
//   the rest                  the runs, one lane group per run (its entries'
//                             (neighbour, vertex) pairs, one load per lane)
__global__ __launch_bounds__(kGatherThreads) void k_bfs_gather(const int2* __restrict__ pairs, int nruns,
                                                               const int4* __restrict__ longrows, int nbig, int nmid,
                                                               const int32_t* __restrict__ col_idx,
                                                               const uint64_t* __restrict__ frontier,
                                                               const uint64_t* __restrict__ mfront,
                                                               const uint64_t* __restrict__ prev2,
                                                               const uint64_t* __restrict__ mprev2,
                                                               ulonglong2* __restrict__ slot,
                                                               uint64_t* __restrict__ mout,
                                                               int32_t* __restrict__ flags, int level, int base) {
  __shared__ ulonglong2 wor[kGatherWaves][kGatherLanes];
  if (flags[level - 1] == 0) return;  // the search of this sweep has ended
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, grp = lane / kGatherLanes, wl = lane % kGatherLanes;
  const ulonglong2* __restrict__ F = reinterpret_cast<const ulonglong2*>(frontier);
  const ulonglong2* __restrict__ P2 = reinterpret_cast<const ulonglong2*>(prev2);
  const int nmid_blocks = (nmid + kGatherWaves - 1) / kGatherWaves;
  if ((int)blockIdx.x < nbig) {
    const int4 lr = longrows[blockIdx.x];  // (vertex, first CSR entry, degree, 0)
    uint64_t a0 = 0ull, a1 = 0ull;
    for (int e0 = wave * kWaveEntries; e0 < lr.z; e0 += kGatherWaves * kWaveEntries)
      row_chunk_or(F, mfront, col_idx, lr.y, lr.z, e0, lane, grp, wl, level, base, a0, a1);
    groups_or(a0, a1);
    if (grp == 0) wor[wave][wl] = make_ulonglong2(a0, a1);
    __syncthreads();
    bool found = false;
    if (wave == 0 && grp == 0) {
#pragma unroll
      for (int w = 1; w < kGatherWaves; ++w) {
        a0 |= wor[w][wl].x;
        a1 |= wor[w][wl].y;
      }
      bfs_settle(F, mfront, P2, mprev2, slot, mout, lr.x, wl, level, base, a0, a1, found);
    }
    raise_flag(found, flags, level);
    return;
  }
  if ((int)blockIdx.x < nbig + nmid_blocks) {
    const int k = ((int)blockIdx.x - nbig) * kGatherWaves + wave;
    if (k >= nmid) return;
    const int4 lr = longrows[nbig + k];
    uint64_t a0 = 0ull, a1 = 0ull;
    for (int e0 = 0; e0 < lr.z; e0 += kWaveEntries)
      row_chunk_or(F, mfront, col_idx, lr.y, lr.z, e0, lane, grp, wl, level, base, a0, a1);
    groups_or(a0, a1);
    bool found = false;
    if (grp == 0) bfs_settle(F, mfront, P2, mprev2, slot, mout, lr.x, wl, level, base, a0, a1, found);
    raise_flag(found, flags, level);
    return;
  }
  const int r = (((int)blockIdx.x - nbig - nmid_blocks) * kGatherWaves + wave) * kGatherGroups + grp;
  // lane wl < kGatherRun of the group holds the run's entry wl: (neighbour, vertex), or (-1, -1)
  const int2 pr = r < nruns && wl < kGatherRun ? pairs[(size_t)r * kGatherRun + wl] : make_int2(-1, -1);
  const int vj = pr.y, uj = pr.x;
  // the entries' chunks (a row's entries are combined below)
  uint64_t c0[kGatherRun], c1[kGatherRun];
  frontier_or(F, uj, entry_mask(mfront, uj, level), kGatherLanes * grp, wl, level, base, c0, c1);
  int cur = -1;
  uint64_t a0 = 0ull, a1 = 0ull;
  bool found = false;
#pragma unroll
  for (int j = 0; j < kGatherRun; ++j) {
    const int v = __builtin_amdgcn_readlane(vj, kGatherLanes * grp + j);
    if (v != cur) {
      if (cur >= 0) bfs_settle(F, mfront, P2, mprev2, slot, mout, cur, wl, level, base, a0, a1, found);
      cur = v;
      a0 = a1 = 0ull;
    }
    a0 |= c0[j];
    a1 |= c1[j];
  }
  if (cur >= 0) bfs_settle(F, mfront, P2, mprev2, slot, mout, cur, wl, level, base, a0, a1, found);
  raise_flag(found, flags, level);
}

// The runs' entries as the gather reads them: lane j of run r gets
// pairs[16 r + j] = (col_idx[e], row of e) for e = first + j below first + count,
// else (-1, -1).  runs[r] = (first CSR entry, count, row of the first entry, 0).
__global__ __launch_bounds__(256) void k_bfs_pairs(const int4* __restrict__ runs, int nruns,
                                                   const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, int2* __restrict__ pairs) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= (size_t)nruns * kGatherRun) return;
  const int4 rd = runs[q / kGatherRun];
  const int j = (int)(q % kGatherRun);
  int2 out = make_int2(-1, -1);
  if (j < rd.y) {
    const int64_t e = (int64_t)rd.x + j;
    int v = rd.z;
    while (row_ptr[v + 1] <= e) ++v;  // the run's rows and the empty rows between them
    out = make_int2(col_idx[e], v);
  }
  pairs[q] = out;
}

// W_v = the sum of the store kernels' partials wq[kq][v] over the sixteen word
// blocks kq, in order.
__global__ __launch_bounds__(256) void k_weights_from_partials(const double* __restrict__ wq, double* __restrict__ W,
                                                               int n, int n_pad) {
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v >= n_pad) return;
  double s = 0.0;
  if (v < n)
    for (int kq = 0; kq < kBfsWords / kStoreWords; ++kq) s += wq[(size_t)kq * n_pad + v];
  W[v] = s;
}

// Flag rows of `sweeps` sweeps: flags[s][0] = 1 (the sources), the rest 0.
__global__ __launch_bounds__(256) void k_bfs_flags(int32_t* __restrict__ flags, int sweeps, int stride) {
  const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (q < (size_t)sweeps * stride) flags[q] = (q % stride) == 0 ? 1 : 0;
}

// Bit b of the nibble to bit 0 of byte b.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) { return ((nib & 0xfu) * 0x00204081u) & 0x01010101u; }

// Levels l0..l1 (one batch, l1 - l0 < 16) into d.  Workgroup: row block rb,
// words 8 kq .. 8 kq + 7 of the sweep; the word blocks of one 128-byte line
// are consecutive workgroups of one XCD (workgroups are handed to the XCDs in
// turn), so the line is fetched into that XCD's L2 once.
// Also the pairs' weights: each row's sum of d^-2 over the found pairs of its
// 8 words (the sources at level l count popcount / l^2, levels from
// count_from on) is added into wq[kq][v], one partial per word block, by one
// thread in a fixed order, so W = sum over kq of wq is the same on every run.
__global__ __launch_bounds__(256) void k_bfs_store(const uint64_t* __restrict__ slots, size_t slot_words,
                                                   const uint64_t* __restrict__ masks,
                                                   const int32_t* __restrict__ flags, uint8_t* __restrict__ d,
                                                   double* __restrict__ wq, int n, int n_pad, int ng, int base,
                                                   int l0, int l1, int count_from) {
  if (l0 > 1 && flags[l0] == 0) return;  // nothing found in this batch; the first batch writes every byte
  __shared__ uint64_t planes[5][kRowBlock][kStoreWords + 1];
  // on XCD x: (rb, kq) = (0, 2 x), (0, 2 x + 1), (1, 2 x), ... for 16 word blocks
  constexpr int kLinesPerXcd = kBfsWords / kStoreWords / kStoreBlocksPerLine / kXcds;
  const int xi = (int)(blockIdx.x / kXcds), x = (int)(blockIdx.x % kXcds);
  const int per_rb = kLinesPerXcd * kStoreBlocksPerLine;
  const int rb = xi / per_rb,
            kq = ((xi % per_rb) / kStoreBlocksPerLine * kXcds + x) * kStoreBlocksPerLine + xi % kStoreBlocksPerLine;
  const int t = threadIdx.x;
  // the batch's levels l0 .. l0 + nl - 1 that found something (the levels after
  // an empty one found nothing)
  int nl = 0;
  while (l0 + nl <= l1 && flags[l0 + nl] != 0) ++nl;
  // planes 0..3: bits of l - l0; plane 4: found in this batch
#pragma unroll
  for (int r = 0; r < kRowBlock * kStoreWords / 256; ++r) {
    const int p = t + 256 * r;
    const int row = p / kStoreWords, kk = p % kStoreWords;
    const int v = rb * kRowBlock + row;
    const size_t q = (size_t)v * kBfsWords + kq * kStoreWords + kk;
    const int chunk = (kq * kStoreWords + kk) / 2;
    uint64_t P0 = 0, P1 = 0, P2 = 0, P3 = 0, Fd = 0;
    double ws = 0.0;
    // every mask first, then the words whose chunk bit is set: all loads in
    // flight at once (a clear lane leaves its load register unwritten)
    uint64_t mk[kBfsSlots], w[kBfsSlots];
    bool on[kBfsSlots];
#pragma unroll
    for (int i = 0; i < kBfsSlots; ++i)
      mk[i] = i < nl ? masks[(size_t)((l0 + i) % kBfsSlots) * n + (v < n ? v : n - 1)] : 0ull;
#pragma unroll
    for (int i = 0; i < kBfsSlots; ++i) {
      on[i] = (v < n) & (((mk[i] >> chunk) & 1ull) != 0ull);
      if (on[i]) w[i] = slots[(size_t)((l0 + i) % kBfsSlots) * slot_words + q];
    }
#pragma unroll
    for (int i = 0; i < kBfsSlots; ++i) {
      const uint64_t nw = on[i] ? w[i] : 0ull;
      Fd |= nw;
      if (i & 1) P0 |= nw;
      if (i & 2) P1 |= nw;
      if (i & 4) P2 |= nw;
      if (i & 8) P3 |= nw;
      const int l = l0 + i;
      if (i < nl && l >= count_from) ws += (double)__popcll(nw) / ((double)l * (double)l);
    }
    // the row's kStoreWords threads are consecutive lanes: add their sums in a fixed tree
#pragma unroll
    for (int m = kStoreWords / 2; m > 0; m >>= 1) ws += __shfl_xor(ws, m, kStoreWords);
    if (kk == 0 && v < n && ws != 0.0) wq[(size_t)kq * n_pad + v] += ws;
    planes[0][row][kk] = P0;
    planes[1][row][kk] = P1;
    planes[2][row][kk] = P2;
    planes[3][row][kk] = P3;
    planes[4][row][kk] = Fd;
  }
  __syncthreads();
  const int wave = t >> 6, row = t & 63;
  const uint32_t lvl = (uint32_t)l0 * 0x01010101u;
#pragma unroll
  for (int r = 0; r < kStoreWords / 4; ++r) {
    const int kk = (kStoreWords / 4) * wave + r;
    const int k = kq * kStoreWords + kk;
    const uint64_t P0 = planes[0][row][kk], P1 = planes[1][row][kk], P2 = planes[2][row][kk],
                   P3 = planes[3][row][kk], Fd = planes[4][row][kk];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int cg = (base + 64 * k + 16 * c) / kColGroup;
      if (cg >= ng) break;  // columns past the padded size
      uint32_t val[4], msk[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int sh = 16 * c + 4 * m;
        const uint32_t x = spread4((uint32_t)(P0 >> sh)) | (spread4((uint32_t)(P1 >> sh)) << 1) |
                           (spread4((uint32_t)(P2 >> sh)) << 2) | (spread4((uint32_t)(P3 >> sh)) << 3);
        msk[m] = spread4((uint32_t)(Fd >> sh)) * 0xffu;
        val[m] = (x + lvl) & msk[m];  // l0 + offset <= 255 in every byte: no carry
      }
      uint4* chunk = reinterpret_cast<uint4*>(d + ((size_t)rb * ng + cg) * kTileBytes + (size_t)row * kColGroup);
      if (l0 == 1) {
        *chunk = make_uint4(val[0], val[1], val[2], val[3]);
      } else if ((Fd >> (16 * c)) & 0xffffull) {
        const uint4 o = *chunk;
        *chunk = make_uint4(val[0] | (o.x & ~msk[0]), val[1] | (o.y & ~msk[1]), val[2] | (o.z & ~msk[2]),
                            val[3] | (o.w & ~msk[3]));
      }
    }
  }
}

// W_i = sum_j d_ij^-2 in double: each wave sums its row block over one column
// slice (columns in ascending order, the tile stream of the force pass), then
// k_weights_sum adds the slices in slice order.
template <bool FD>
__global__ __launch_bounds__(256) void k_weights(const uint8_t* __restrict__ d, const float* __restrict__ df,
                                                 double* __restrict__ wpart, int nrb, int ng, int gps, int n_pad) {
  __shared__ double lut[256];
  if constexpr (!FD) {
    lut[threadIdx.x] = threadIdx.x ? 1.0 / ((double)threadIdx.x * (double)threadIdx.x) : 0.0;
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int rb = blockIdx.x * 4 + wave;
  if (rb >= nrb) return;
  const int g0 = blockIdx.y * gps, g1 = min(g0 + gps, ng);
  double s = 0.0;
  if (g0 < g1) {
    auto q = load_chunk<FD>(d, df, rb, ng, g0, lane);
    for (int g = g0; g < g1; ++g) {
      const auto qn = load_chunk<FD>(d, df, rb, ng, min(g + 1, g1 - 1), lane);
#pragma unroll
      for (int k = 0; k < kColGroup; ++k) {
        if constexpr (FD) {
          const double dv = (double)fchunk_at(q, k);
          s += dv > 0.0 ? 1.0 / (dv * dv) : 0.0;
        } else {
          s += lut[byte_of(chunk_word(q, k), k & 3)];
        }
      }
      q = qn;
    }
  }
  wpart[(size_t)blockIdx.y * n_pad + rb * kRowBlock + lane] = s;
}

__global__ __launch_bounds__(256) void k_weights_sum(const double* __restrict__ wpart, int slices, double* __restrict__ W,
                                                     int n, int n_pad) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n_pad) return;
  const double s = sum_strided(wpart + i, slices, (size_t)n_pad);
  W[i] = i < n ? s : 0.0;
}

}  // namespace

int bfs_sources_per_sweep() { return kBfsSources; }
int bfs_words() { return kBfsWords; }
int bfs_slots() { return kBfsSlots; }

int bfs_run_entries() { return kGatherRun; }

hipError_t launch_bfs_flags(int32_t* flags, int sweeps, int stride, hipStream_t s) {
  const size_t q = (size_t)sweeps * stride;
  if (q == 0) return hipSuccess;
  k_bfs_flags<<<blocks_for(q), 256, 0, s>>>(flags, sweeps, stride);
  return hipGetLastError();
}

hipError_t launch_weights_from_partials(const double* wq, double* W, int n, int n_pad, hipStream_t s) {
  k_weights_from_partials<<<blocks_for(n_pad), 256, 0, s>>>(wq, W, n, n_pad);
  return hipGetLastError();
}

int bfs_weight_partials() { return kBfsWords / kStoreWords; }

int bfs_mid_max_degree() { return kMidMax; }

hipError_t launch_bfs_pairs(const int4* runs, int nruns, const int64_t* row_ptr, const int32_t* col_idx, int2* pairs,
                            hipStream_t s) {
  if (nruns <= 0) return hipSuccess;
  k_bfs_pairs<<<blocks_for((size_t)nruns * kGatherRun), 256, 0, s>>>(runs, nruns, row_ptr, col_idx, pairs);
  return hipGetLastError();
}

hipError_t launch_bfs_level(const int2* pairs, int nruns, const int4* longrows, int nbig, int nmid,
                            const int32_t* col_idx, const uint64_t* slots, uint64_t* masks, int n, int base,
                            int level, int32_t* flags, hipStream_t s) {
  if (n <= 0 || nruns + nbig + nmid == 0) return hipSuccess;
  const size_t words = (size_t)n * kBfsWords;
  const int s1 = (level - 1) % kBfsSlots, s2 = (level + kBfsSlots - 2) % kBfsSlots, s0 = level % kBfsSlots;
  const uint64_t* frontier = slots + (size_t)s1 * words;
  const uint64_t* prev2 = slots + (size_t)s2 * words;  // read from level 3 on
  uint64_t* out = const_cast<uint64_t*>(slots) + (size_t)s0 * words;
  const int per_block = kGatherWaves * kGatherGroups;
  const unsigned blocks = (unsigned)(nbig + (nmid + kGatherWaves - 1) / kGatherWaves + (nruns + per_block - 1) / per_block);
  k_bfs_gather<<<blocks, kGatherThreads, 0, s>>>(pairs, nruns, longrows, nbig, nmid, col_idx, frontier,
                                                 masks + (size_t)s1 * n, prev2, masks + (size_t)s2 * n,
                                                 reinterpret_cast<ulonglong2*>(out), masks + (size_t)s0 * n, flags,
                                                 level, base);
  return hipGetLastError();
}

hipError_t launch_bfs_store(const uint64_t* slots, const uint64_t* masks, const int32_t* flags, uint8_t* d,
                            double* wq, int n, int n_pad, int base, int l0, int l1, int count_from, hipStream_t s) {
  if (n <= 0 || l1 < l0) return hipSuccess;
  const int nrb = n_pad / kRowBlock;
  k_bfs_store<<<(unsigned)nrb * (kBfsWords / kStoreWords), 256, 0, s>>>(
      slots, (size_t)n * kBfsWords, masks, flags, d, wq, n, n_pad, n_pad / kColGroup, base, l0, l1, count_from);
  return hipGetLastError();
}

hipError_t launch_weights(const uint8_t* d, const float* df, double* W, double* wpart, const Split& sp, int n,
                          hipStream_t s) {
  const int n_pad = sp.nrb * kRowBlock;
  const dim3 grid(sp.blocks_x, sp.slices);
  if (df) k_weights<true><<<grid, 256, 0, s>>>(d, df, wpart, sp.nrb, sp.ng, sp.groups_per_slice, n_pad);
  else k_weights<false><<<grid, 256, 0, s>>>(d, df, wpart, sp.nrb, sp.ng, sp.groups_per_slice, n_pad);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_weights_sum<<<blocks_for(n_pad), 256, 0, s>>>(wpart, sp.slices, W, n, n_pad);
  return hipGetLastError();
}

}  // namespace sl
