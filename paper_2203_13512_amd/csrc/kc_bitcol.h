// kc_bitcol.h -- BitCol device code shared by the translation units of the
// listing kernels (kc_bitcol.hip: word classes of 1 to 16 words and the host
// side; kc_bitcol_wide.hip: the classes of 24 to 64 words), so that the many
// kernel instances compile in parallel.  The method is described in
// kc_bitcol.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "kc_internal.h"

#define KC_NCLASS 10
static const int kWClass[KC_NCLASS] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 64};
// The widest classes keep their bitmaps in device memory while listing
// (ListLayout GB): 48 and 64 words always, 24 and 32 words with per-vertex
// output; their staging builds the local adjacency matrix in device memory.
static inline bool class_in_device_memory(int cls, bool pv) { return cls >= 8 || (pv && cls >= 6); }
// Largest k at which those classes run (see kc_list_bitcol).
#define KC_DEVMEM_KMAX 5

static inline int wclass_of(int s) {
  int w = (s + 31) / 32;
  for (int c = 0; c < KC_NCLASS; ++c)
    if (w <= kWClass[c]) return c;
  return -1;
}
__device__ __forceinline__ int d_wclass_of(int s) {
  int w = (s + 31) >> 5;
  if (w <= 1) return 0;
  if (w <= 2) return 1;
  if (w <= 4) return 2;
  if (w <= 8) return 3;
  if (w <= 12) return 4;
  if (w <= 16) return 5;
  if (w <= 24) return 6;
  if (w <= 32) return 7;
  if (w <= 48) return 8;
  if (w <= 64) return 9;
  return -1;
}
__device__ __forceinline__ int d_wclass_words(int c) {
  const int t[KC_NCLASS] = {1, 2, 4, 8, 12, 16, 24, 32, 48, 64};
  return t[c];
}

struct RootInfo {
  int32_t* s;        // [R] local size
  int32_t* cls;      // [R] word class
  int64_t* boff;     // [R] word offset of the root's bitmaps
  int64_t* poff;     // [R] position offset (perm/color)
};

// ============================================================== staging
struct StageArgs {
  const int32_t* drp;
  const int32_t* dcol;
  const int32_t* roots;
  const int32_t* core;
  RootInfo ri;
  uint32_t* B;
  uint32_t* Bin;      // per-vertex mode only
  int32_t* perm;
  uint16_t* color;
  float* features;    // [R x 4] (d+, core, colors, |E_u|)
  unsigned long long* stage_bytes;
  int* flags;
};

__device__ __forceinline__ int lds_lower_bound(const int32_t* a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ int lds_upper_bound(const int32_t* a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Dynamic LDS layout for a stage workgroup with class words WM (S = 32*WM):
//   ids[S] i32 | off[S+1] i32 | deg[S] i32 | order[S] i32 | color[S] i32 |
//   pos[S] i32 | used[WM+2] u32 | M1[WM*S] u32 | M2[WM*S] u32 (per-vertex)
// With `mat` (device memory, WM*S words per matrix and workgroup) the two
// matrices live there instead of in LDS.
static size_t stage_lds_bytes(int WM, bool pv, bool mat_in_lds = true) {
  size_t S = 32 * (size_t)WM;
  return 4 * (S + S + 1 + S + S + S + S + WM + 2) + (mat_in_lds ? 4 * (size_t)WM * S * (pv ? 2 : 1) : 0) + 64;
}

// Barrier of a staging workgroup.  With the matrices in device memory the
// bit sets are built by atomics in L2, so the barrier is followed by an
// acquire at device scope: later loads do not hit stale lines of the CU's
// vector cache.
__device__ __forceinline__ void stage_sync(const uint32_t* mat) {
  __syncthreads();
  if (mat) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <bool PV>
__global__ __launch_bounds__(64) void k_bitcol_stage(StageArgs a, const int32_t* __restrict__ list, int32_t nlist,
                                                     int WM, uint32_t* mat) {
  extern __shared__ uint32_t lds[];
  const int S = 32 * WM;
  int32_t* ids = (int32_t*)lds;
  int32_t* off = ids + S;
  int32_t* deg = off + S + 1;
  int32_t* order = deg + S;
  int32_t* color = order + S;
  int32_t* pos = color + S;
  uint32_t* used = (uint32_t*)(pos + S);
  uint32_t* M1 = mat ? mat + (size_t)blockIdx.x * (PV ? 2 : 1) * WM * S : used + WM + 2;
  uint32_t* M2 = M1 + (size_t)WM * S;
  const int lane = threadIdx.x;

  uint64_t staged_bytes = 0;  // lane 0: algorithmic bytes of the roots this workgroup staged
  for (int32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int32_t r = list[li];
    const int32_t u = a.roots[r];
    const int32_t s = a.ri.s[r];
    const int Wc = d_wclass_words(a.ri.cls[r]);
    const int Sr = 32 * Wc;  // positions of this root (<= S)
    const int32_t base = a.drp[u];
    // ids and out-degrees of the local vertices
    for (int i = lane; i < S; i += 64) {
      if (i < s) {
        int32_t v = a.dcol[base + i];
        ids[i] = v;
        deg[i] = a.drp[v + 1] - a.drp[v];
      }
      color[i] = 0;
    }
    for (int i = lane; i < WM * S; i += 64) {
      M1[i] = 0;
      if (PV) M2[i] = 0;
    }
    stage_sync(mat);
    // off = exclusive prefix of deg over i < s (wave scan in chunks of 64)
    {
      int carry = 0;
      for (int c0 = 0; c0 < s; c0 += 64) {
        int i = c0 + lane;
        int x = i < s ? deg[i] : 0;
        int incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          int y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        if (i < s) off[i] = carry + incl - x;
        carry += __shfl(incl, 63, 64);
      }
      if (lane == 0) off[s] = carry;
    }
    stage_sync(mat);
    const int32_t T = off[s];
    // pass 1: undirected adjacency of G_u in local (id) order
    unsigned edges = 0;
    for (int32_t t0 = 0; t0 < T; t0 += 64) {
      int32_t t = t0 + lane;
      bool hit = false;
      if (t < T) {
        int i = lds_upper_bound(off, s + 1, t) - 1;
        int32_t v = ids[i];
        int32_t x = a.dcol[a.drp[v] + (t - off[i])];
        int j = lds_lower_bound(ids, s, x);
        if (j < s && ids[j] == x) {
          hit = true;
          atomicOr(&M1[(j >> 5) * S + i], 1u << (j & 31));
          atomicOr(&M1[(i >> 5) * S + j], 1u << (i & 31));
        }
      }
      edges += (unsigned)__popcll(kc_ballot(hit));
    }
    stage_sync(mat);
    // local degrees
    for (int i = lane; i < s; i += 64) {
      int d = 0;
      for (int w = 0; w < Wc; ++w) d += __popc(M1[w * S + i]);
      deg[i] = d;
    }
    stage_sync(mat);
    // coloring order: degree descending, then id (= local index) ascending
    for (int i = lane; i < s; i += 64) {
      int di = deg[i], rk = 0;
      for (int j = 0; j < s; ++j) {
        int dj = deg[j];
        rk += (dj > di) || (dj == di && j < i);
      }
      order[rk] = i;
    }
    stage_sync(mat);
    // greedy coloring, one vertex at a time
    const int Wu = (s + 1 + 31) / 32;
    int maxc = 0;
    for (int t = 0; t < s; ++t) {
      const int v = order[t];
      for (int w = lane; w < Wu; w += 64) used[w] = 0;
      stage_sync(mat);
      for (int j = lane; j < s; j += 64) {
        if ((M1[(j >> 5) * S + v] >> (j & 31)) & 1u) {
          int c = color[j];
          if (c > 0) atomicOr(&used[c >> 5], 1u << (c & 31));
        }
      }
      stage_sync(mat);
      int found = 0x7fffffff;
      for (int w0 = 0; w0 < Wu; w0 += 64) {
        int w = w0 + lane;
        uint32_t m = w < Wu ? ~used[w] : 0u;
        if (w == 0) m &= ~1u;  // colors start at 1
        uint64_t b = kc_ballot(m != 0u);
        if (b) {
          int fl = __ffsll((long long)b) - 1;
          uint32_t mm = (uint32_t)__shfl((int)m, fl, 64);
          found = (w0 + fl) * 32 + __ffs(mm) - 1;
          break;
        }
      }
      if (lane == 0) color[v] = found;
      maxc = found > maxc ? found : maxc;
      stage_sync(mat);
    }
    // positions sorted by (color, local index)
    for (int i = lane; i < s; i += 64) {
      int ci = color[i], p = 0;
      for (int j = 0; j < s; ++j) {
        int cj = color[j];
        p += (cj < ci) || (cj == ci && j < i);
      }
      pos[i] = p;
      order[p] = i;  // inverse permutation
    }
    for (int i = lane; i < WM * S; i += 64) M1[i] = 0;
    stage_sync(mat);
    // pass 2: encoded bitmaps in color order
    for (int32_t t0 = 0; t0 < T; t0 += 64) {
      int32_t t = t0 + lane;
      if (t < T) {
        int i = lds_upper_bound(off, s + 1, t) - 1;
        int32_t v = ids[i];
        int32_t x = a.dcol[a.drp[v] + (t - off[i])];
        int j = lds_lower_bound(ids, s, x);
        if (j < s && ids[j] == x) {
          int pi = pos[i], pj = pos[j];
          int hi = color[j] < color[i] ? pi : pj;  // higher color: owner of the out-bitmap
          int lo = color[j] < color[i] ? pj : pi;
          atomicOr(&M1[(lo >> 5) * S + hi], 1u << (lo & 31));
          if (PV) atomicOr(&M2[(hi >> 5) * S + lo], 1u << (hi & 31));
        }
      }
    }
    stage_sync(mat);
    // write out (column-major, Sr positions per word row)
    const int64_t bo = a.ri.boff[r];
    for (int w = 0; w < Wc; ++w)
      for (int p = lane; p < Sr; p += 64) {
        a.B[bo + (int64_t)w * Sr + p] = M1[w * S + p];
        if (PV) a.Bin[bo + (int64_t)w * Sr + p] = M2[w * S + p];
      }
    const int64_t po = a.ri.poff[r];
    for (int p = lane; p < Sr; p += 64) {
      if (p < s) {
        int i = order[p];
        a.perm[po + p] = ids[i];
        a.color[po + p] = (uint16_t)color[i];
      } else {
        a.perm[po + p] = -1;
        a.color[po + p] = 0;
      }
    }
    if (lane == 0) {
      if (a.features) {
        a.features[4 * (int64_t)r + 0] = (float)s;
        a.features[4 * (int64_t)r + 1] = a.core ? (float)a.core[u] : 0.0f;
        a.features[4 * (int64_t)r + 2] = (float)maxc;
        a.features[4 * (int64_t)r + 3] = (float)edges;
      }
      staged_bytes += 4ull * ((uint64_t)s + (uint64_t)T);
    }
    stage_sync(mat);
  }
  // one atomic per workgroup for the staging counter, not one per root
  if (lane == 0 && staged_bytes) atomicAdd(a.stage_bytes, (unsigned long long)staged_bytes);
}

// ============================================================== listing
struct ListArgs {
  const int32_t* roots;
  RootInfo ri;
  const uint32_t* B;
  const uint32_t* Bin;
  const int32_t* perm;
  const uint16_t* color;
  const uint64_t* tasks;   // (root << 32) | ((v1 + 1) << 16) | (v2 + 1)
  int64_t ntasks;
  unsigned long long* head;  // queue head
  int chunk;
  int k;
  const int32_t* vk;                 // per-vertex k (nullable)
  unsigned long long* root_count;    // per-root attribution (nullable)
  int cmax;   // re-encode sets of at most cmax members (0 = never)
  int clev;   // ... at nodes of level >= clev
  int noprune;  // ablation: every position counts as color >= any level (no color prune)
  unsigned long long* count;
  unsigned long long* pv;
  unsigned long long* counters;  // nodes, isect, work, wave-wide joins, joins on re-encoded rows
  uint64_t* root_work;
  uint64_t* root_isect;
  int* flags;
};

// LDS layout of a listing workgroup (offsets in 32-bit words, 64-bit
// fields on even offsets):
//   B[W][S+1] | Bin[W][S+1] (per-vertex) | color[S] | firstpos[KMAX+2] |
//   C0[W] | shared scalars[16] | NW wave blocks | cnt[S] u64 (per-vertex)
// A wave block (sized for K = k+1 levels at run time) holds tot[K] u64 |
// cur[K] | chosen[K] | stack[K][W] | a region used by one evaluation at a
// time: the candidate list of a level-3 node, or a re-encoded node.
#define KC_KMAX 32

// GB: the root's bitmaps are read in place from device memory (the staged
// column-major block, row stride S) instead of being copied into LDS -- the
// layout of local subgraphs too large for LDS (48 and 64 words, and the
// per-vertex classes above 16 words, whose in-neighbour bitmaps double it).
template <int W, int NW, bool PV, bool COMP, bool GB = false>
struct ListLayout {
  static constexpr int S = 32 * W;
  static constexpr int SP = GB ? S : S + 1;  // row stride (in LDS, S + 1 keeps accesses bank-conflict free)
  static constexpr int a2(int x) { return (x + 1) & ~1; }
  static constexpr int a4(int x) { return (x + 3) & ~3; }
  static constexpr int oB = 0;
  static constexpr int oBin = oB + (GB ? 0 : W * SP);
  static constexpr int oCol = oBin + (PV && !GB ? W * SP : 0);
  static constexpr int oFirst = oCol + S;
  static constexpr int oC0 = oFirst + KC_KMAX + 2;
  static constexpr int oSh = a2(oC0 + W);
  static constexpr int oWave = a4(oSh + 16);
  // Two-word re-encoding (sets of 65..128 members) is used when counting.
  static constexpr bool C2 = COMP && !PV && W >= 4 && W <= 16;
  // Per-wave region used by one evaluation at a time: the candidate list of a
  // lane-parallel level-3 node, or a re-encoded node (rows, queue or in-rows,
  // color masks, member list).
  static constexpr int U1 = 2 * (64 + 128 + 12) + 32;        // one-word rows
  static constexpr int U2 = 4 * 128 + 4 * 128 + 4 * 12 + 64;  // two-word rows
  static constexpr int UW = a4(S / 2 > (C2 ? U2 : (COMP ? U1 : 0)) ? S / 2 : (C2 ? U2 : (COMP ? U1 : 0)));
  // per wave, for recursion depth K = k + 1 (runtime):
  //   tot[K] u64 | cur[K] | chosen[K] | stack[K][W] | (16-byte aligned) region[UW]
  __host__ __device__ static constexpr int oU(int K) { return a4(2 * K + 2 * K + K * W); }
  __host__ __device__ static constexpr int wave_words(int K) { return oU(K) + UW; }
  __host__ __device__ static constexpr int oCnt(int K) { return oWave + NW * wave_words(K); }
  __host__ __device__ static constexpr int words(int K) { return oCnt(K) + (PV ? 2 * S : 0); }
  static size_t bytes(int K) { return 4 * (size_t)words(K); }
};

// Wave-wide popcount of a lane-split bitmap (lane i < W holds word i).
__device__ __forceinline__ uint32_t split_popc(uint32_t w) { return kc_wave_sum_u32((uint32_t)__popc(w)); }

// First member of the lane-split set `w` at a position >= from, or -1.
template <int W>
__device__ __forceinline__ int split_next(uint32_t w, int from, int lane) {
  int fw = from >> 5;
  uint32_t m = 0;
  if (lane < W) {
    m = w;
    if (lane < fw) m = 0;
    else if (lane == fw) m &= (~0u) << (from & 31);
  }
  uint64_t b = kc_ballot(m != 0u);
  if (!b) return -1;
  int fl = __ffsll((long long)b) - 1;
  uint32_t mm = kc_readlane(m, fl);
  return fl * 32 + __ffs(mm) - 1;
}

// Level-2 node with set C (lane-split word in `cw`): returns the node's leaf
// count (wave-uniform) and adds the BitJoins performed to `joins`.
template <int W, bool PV, int SP>
__device__ __forceinline__ uint64_t leaf_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                              int s, int first2, uint32_t cw, int lane, uint64_t& joins,
                                              unsigned long long* cnt, int chunk0 = 0, int chunk_step = 1) {
  // highest nonzero word bounds the scan
  int hiw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
  if (hiw < 0) return 0;
  uint32_t c[W];
#pragma unroll
  for (int i = 0; i < W; ++i) c[i] = kc_readlane(cw, i);
  const int end = (hiw + 1) * 32 < s ? (hiw + 1) * 32 : s;
  uint32_t total = 0;
  uint32_t nj = 0;
  const int start = (PV ? 0 : (first2 & ~63)) + 64 * chunk0;
  for (int p0 = start; p0 < end; p0 += 64 * chunk_step) {
    const int p = p0 + lane;
    uint32_t word = (uint32_t)__shfl((int)cw, (p >> 5) & 63, 64);
    bool mem = p < end && ((word >> (p & 31)) & 1u);
    bool join = mem && p >= first2;
    uint32_t acc = 0, acc_in = 0;
    if (join) {
#pragma unroll
      for (int i = 0; i < W; ++i) {
        if (i > hiw) break;
        acc += (uint32_t)__popc(Bl[i * SP + p] & c[i]);
      }
    }
    if (PV && mem) {
#pragma unroll
      for (int i = 0; i < W; ++i) {
        if (i > hiw) break;
        acc_in += (uint32_t)__popc(Bil[i * SP + p] & c[i]);
      }
      uint32_t add = acc + acc_in;
      if (add) atomicAdd(&cnt[p], (unsigned long long)add);
    }
    total += acc;
    nj += (uint32_t)__popcll(kc_ballot(join));
  }
  joins += nj;
  return (uint64_t)kc_wave_sum_u32(total);
}

// Level-3 node with set C (lane-split word in `cw`), evaluated lane-parallel:
// the members v of C with color >= 3 are compacted into `vlist` and dealt to
// lanes (passes part, part+nparts, ... of 64); each lane forms C' = B(v) & C
// in registers and, when |C'| >= 2, walks the members w of C' with color >= 2
// itself, adding popcount(B(w) & C') (B(w) only has bits below w, so only the
// words up to w's own word are read).  This is BitColList at l = 3 and l = 2
// with the same pruning and join count, without wave-wide steps per node.
// Returns this lane's share of the node's leaves; joins/nodes are per lane.
template <int W, bool PV, int SP>
__device__ __forceinline__ uint64_t level3_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                                int s, int first2, int first3, uint32_t cw, int lane,
                                                uint16_t* __restrict__ vlist, uint64_t& joins, uint64_t& nodes,
                                                unsigned long long* cnt, int part, int nparts) {
  const int hiw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
  if (hiw < 0) return 0;
  uint32_t c[W];
#pragma unroll
  for (int i = 0; i < W; ++i) c[i] = kc_readlane(cw, i);
  const int end = (hiw + 1) * 32 < s ? (hiw + 1) * 32 : s;
  int mcount = 0;
  for (int p0 = first3 & ~63; p0 < end; p0 += 64) {
    const int p = p0 + lane;
    const uint32_t word = (uint32_t)__shfl((int)cw, (p >> 5) & 63, 64);
    const bool mem = p >= first3 && p < end && ((word >> (p & 31)) & 1u);
    const uint64_t mk = kc_ballot(mem);
    if (mem) vlist[mcount + kc_mbcnt(mk)] = (uint16_t)p;
    mcount += __popcll(mk);
  }
  kc_wave_lds_sync();
  const int f2w = first2 >> 5;
  const uint32_t f2m = (~0u) << (first2 & 31);
  uint64_t total = 0;
  for (int base = part * 64; base < mcount; base += 64 * nparts) {
    const int idx = base + lane;
    if (idx >= mcount) continue;
    const int v = vlist[idx];
    joins++;
    uint32_t cv[W];
    int pc = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      cv[i] = i <= hiw ? (Bl[i * SP + v] & c[i]) : 0u;
      pc += __popc(cv[i]);
    }
    if (pc < 2) continue;
    nodes++;
    uint32_t leaf = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      uint32_t m = cv[i];
      if (!PV) m = i < f2w ? 0u : (i == f2w ? (m & f2m) : m);
      while (m) {
        const int b = __ffs(m) - 1;
        m &= m - 1;
        const int w = i * 32 + b;
        uint32_t out = 0;
        if (!PV || w >= first2) {
#pragma unroll
          for (int j = 0; j <= i; ++j) out += (uint32_t)__popc(Bl[j * SP + w] & cv[j]);
          joins++;
        }
        leaf += out;
        if (PV) {
          uint32_t in = 0;
#pragma unroll
          for (int j = i; j < W; ++j) in += (uint32_t)__popc(Bil[j * SP + w] & cv[j]);
          if (out + in) atomicAdd(&cnt[w], (unsigned long long)(out + in));
        }
      }
    }
    total += leaf;
    if (PV && leaf) atomicAdd(&cnt[v], (unsigned long long)leaf);
  }
  return total;
}

// ---- compressed nodes ----------------------------------------------------
// Once a node's candidate set C has at most 64 members, the sub-DAG it
// induces is re-encoded: member j (members in position order, which is color
// order) gets the 64-bit row R_j = {j' : member j' is in B(member j)}.  This
// is the out-neighbour reduction of Sec. 7.2 applied to the candidate set:
// every BitJoin below the node becomes one 64-bit AND and popcount, and the
// encoding keeps the color order, so "color >= l" stays a suffix of member
// indices.  Each lane takes one candidate of the node and finishes its
// subtree with a depth-first walk whose levels are unrolled at compile time
// (cdfs<L>), so the walk's sets stay in registers.
#define KC_CMAX 10  // deepest level evaluated on compressed rows
#define KC_QMAX 8   // deepest level evaluated through the level-2 queue (count mode)
#define KC_Q2MAX 5  // the same for two-word rows (children of wide nodes only)

struct CNode {
  const uint64_t* rows;   // R_j (LDS)
  const uint64_t* rins;   // per-vertex: {j' : member j in B(member j')} (LDS)
  const uint16_t* mlist;  // member j -> position
  const uint64_t* cm;     // cm[c] = members with color >= c (LDS, c <= KC_CMAX)
};

template <bool PV, int L>
__device__ __forceinline__ uint64_t cdfs(const uint64_t* __restrict__ rows, const uint64_t* __restrict__ rins,
                                         const uint16_t* __restrict__ mlist, const uint64_t* __restrict__ cm,
                                         uint64_t X, uint64_t& joins, uint64_t& nodes, unsigned long long* cnt) {
  if constexpr (L == 2) {
    uint64_t t = 0;
    const uint64_t c2 = cm[2];
    uint64_t cand = PV ? X : (X & c2);
    while (cand) {
      const int y = __ffsll((long long)cand) - 1;
      cand &= cand - 1;
      uint32_t out = 0;
      if (!PV || ((c2 >> y) & 1ull)) {
        out = (uint32_t)__popcll(rows[y] & X);
        joins++;
      }
      t += out;
      if (PV) {
        const uint32_t in = (uint32_t)__popcll(rins[y] & X);
        if (out + in) atomicAdd(&cnt[mlist[y]], (unsigned long long)(out + in));
      }
    }
    return t;
  } else {
    uint64_t t = 0;
    uint64_t cand = X & cm[L];
    while (cand) {
      const int y = __ffsll((long long)cand) - 1;
      cand &= cand - 1;
      const uint64_t X2 = rows[y] & X;
      joins++;
      if (__popcll(X2) >= L - 1) {
        nodes++;
        const uint64_t sub = cdfs<PV, L - 1>(rows, rins, mlist, cm, X2, joins, nodes, cnt);
        t += sub;
        if (PV && sub) atomicAdd(&cnt[mlist[y]], (unsigned long long)sub);
      }
    }
    return t;
  }
}

// ---- count-only evaluation of compressed nodes of level >= 4 -------------
// Each lane holds its member's row R in registers.  The levels above 3 are
// walked by the whole wave with wave-uniform sets (the scalar unit does the
// set bookkeeping; a chosen member's row is read from its lane); at a level-3
// node every lane z forms its child R_z & X at once, and the children that
// qualify as level-2 nodes are appended to a per-wave queue in LDS.  Each time
// the queue holds 64 nodes every lane evaluates one of them (its leaves are
// the popcounts of the BitJoins at level 2), so the leaf work is spread over
// all lanes however unbalanced the subtrees above are.  Same joins, same
// pruning and same counts as the recursive form.

// Leaves of a level-2 node X: over members y of X with color >= 2, the sum of
// popcount(R_y & X).  R_y only holds members below y, so for y < 32 the high
// word is zero and one 32-bit AND and popcount suffice.
__device__ __forceinline__ uint32_t cleaf(const uint64_t* __restrict__ rows, uint64_t X, uint64_t c2) {
  const uint32_t xl = (uint32_t)X, xh = (uint32_t)(X >> 32);
  const uint64_t cand = X & c2;
  uint32_t lo = (uint32_t)cand, hi = (uint32_t)(cand >> 32);
  const uint32_t* r32 = (const uint32_t*)rows;
  uint32_t acc = 0;
  while (lo) {
    const int y = __ffs((int)lo) - 1;
    lo &= lo - 1;
    acc += (uint32_t)__popc(r32[2 * y] & xl);
  }
  while (hi) {
    const int y = __ffs((int)hi) + 31;
    hi &= hi - 1;
    const uint64_t r = rows[y];
    acc += (uint32_t)__popc((uint32_t)r & xl) + (uint32_t)__popc((uint32_t)(r >> 32) & xh);
  }
  return acc;
}

struct CQueue {
  const uint64_t* rows;  // R_j (LDS)
  uint64_t* q;           // 128 pending level-2 nodes (LDS, per wave)
  int n;                 // pending count (wave-uniform)
  uint64_t c2, c3;       // members with color >= 2, >= 3
  uint64_t acc;          // this lane's leaves
};

__device__ __forceinline__ void cq_eval(CQueue& Q, int lane, int cnt_lanes, uint64_t& joins) {
  kc_wave_lds_sync();
  if (lane < cnt_lanes) {
    const uint64_t Y = Q.q[Q.n - cnt_lanes + lane];
    joins += (uint64_t)__popcll(Y & Q.c2);
    Q.acc += cleaf(Q.rows, Y, Q.c2);
  }
  Q.n -= cnt_lanes;
  kc_wave_lds_sync();
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t readfirstlane64(uint64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <int L>
__device__ __forceinline__ void wdfs(CQueue& Q, const uint64_t* __restrict__ cm, uint64_t R, uint64_t X,
                                     uint64_t top, int lane, uint64_t& joins, uint64_t& nodes) {
  if constexpr (L == 3) {
    // level-3 node: lane z is candidate z (a node without candidates adds
    // nothing: its join and node counts and the queue stay as they are)
    const uint64_t cands = X & Q.c3 & top;
    if (!cands) return;
    const bool cand = (cands >> lane) & 1ull;
    const uint64_t X2 = R & X;
    joins += cand ? 1u : 0u;
    const bool push = cand && __popcll(X2) >= 2;
    nodes += push ? 1u : 0u;
    const uint64_t pm = kc_ballot(push);
    if (push) Q.q[Q.n + kc_mbcnt(pm)] = X2;
    Q.n += __popcll(pm);
    if (Q.n >= 64) cq_eval(Q, lane, 64, joins);
  } else {
    uint64_t cand = X & readfirstlane64(cm[L]) & top;
    while (cand) {
      const int y = __ffsll((long long)cand) - 1;
      cand &= cand - 1;
      const uint64_t X2 = readlane64(R, y) & X;
      joins += (lane == 0);
      if (__popcll(X2) >= L - 1) {
        nodes += (lane == 0);
        wdfs<L - 1>(Q, cm, R, X2, ~0ull, lane, joins, nodes);
      }
    }
  }
}

// ---- count-only evaluation of compressed nodes of 65 to 128 members --------
// Same scheme with two-word sets: lane i holds the row of member i (one word:
// R_i only has members below i) and of member 64+i (two words).  Rows live in
// LDS as four 32-bit words each, the level-2 queue as pairs of 64-bit words.

// Leaves of a level-2 node X = (xl, xh): a member in 32-bit word q of X has
// nonzero row words 0..q only.
__device__ __forceinline__ uint32_t cleaf2(const uint32_t* __restrict__ r, uint64_t xl, uint64_t xh, uint64_t c2l,
                                           uint64_t c2h) {
  const uint32_t x0 = (uint32_t)xl, x1 = (uint32_t)(xl >> 32), x2 = (uint32_t)xh, x3 = (uint32_t)(xh >> 32);
  const uint64_t cl = xl & c2l, ch = xh & c2h;
  uint32_t w0 = (uint32_t)cl, w1 = (uint32_t)(cl >> 32), w2 = (uint32_t)ch, w3 = (uint32_t)(ch >> 32);
  uint32_t acc = 0;
  while (w0) {
    const int y = __ffs((int)w0) - 1;
    w0 &= w0 - 1;
    acc += (uint32_t)__popc(r[4 * y] & x0);
  }
  while (w1) {
    const int y = __ffs((int)w1) + 31;
    w1 &= w1 - 1;
    const uint2 v = *(const uint2*)(r + 4 * y);
    acc += (uint32_t)__popc(v.x & x0) + (uint32_t)__popc(v.y & x1);
  }
  while (w2) {
    const int y = __ffs((int)w2) + 63;
    w2 &= w2 - 1;
    const uint4 v = *(const uint4*)(r + 4 * y);
    acc += (uint32_t)__popc(v.x & x0) + (uint32_t)__popc(v.y & x1) + (uint32_t)__popc(v.z & x2);
  }
  while (w3) {
    const int y = __ffs((int)w3) + 95;
    w3 &= w3 - 1;
    const uint4 v = *(const uint4*)(r + 4 * y);
    acc += (uint32_t)__popc(v.x & x0) + (uint32_t)__popc(v.y & x1) + (uint32_t)__popc(v.z & x2) +
           (uint32_t)__popc(v.w & x3);
  }
  return acc;
}

struct CQueue2 {
  const uint32_t* rows;  // 128 rows x 4 words (LDS)
  uint64_t* q;           // 128 pending level-2 nodes x 2 words (LDS, per wave)
  int n;
  uint64_t c2l, c2h, c3l, c3h;
  uint64_t acc;
};

__device__ __forceinline__ void cq2_eval(CQueue2& Q, int lane, int cnt_lanes, uint64_t& joins) {
  kc_wave_lds_sync();
  if (lane < cnt_lanes) {
    const int e = Q.n - cnt_lanes + lane;
    const uint64_t yl = Q.q[2 * e], yh = Q.q[2 * e + 1];
    joins += (uint64_t)(__popcll(yl & Q.c2l) + __popcll(yh & Q.c2h));
    Q.acc += cleaf2(Q.rows, yl, yh, Q.c2l, Q.c2h);
  }
  Q.n -= cnt_lanes;
  kc_wave_lds_sync();
}

// Appends the qualifying children of the candidates in `cand` (one per lane).
__device__ __forceinline__ void cq2_push(CQueue2& Q, bool cand, uint64_t yl, uint64_t yh, int lane, uint64_t& joins,
                                         uint64_t& nodes) {
  joins += cand ? 1u : 0u;
  const bool push = cand && (__popcll(yl) + __popcll(yh)) >= 2;
  nodes += push ? 1u : 0u;
  const uint64_t pm = kc_ballot(push);
  if (push) {
    const int e = Q.n + kc_mbcnt(pm);
    Q.q[2 * e] = yl;
    Q.q[2 * e + 1] = yh;
  }
  Q.n += __popcll(pm);
  if (Q.n >= 64) cq2_eval(Q, lane, 64, joins);
}

template <int L>
__device__ __forceinline__ void wdfs2(CQueue2& Q, const uint64_t* __restrict__ cm, uint64_t R0, uint64_t R1l,
                                      uint64_t R1h, uint64_t Xl, uint64_t Xh, uint64_t topl, uint64_t toph, int lane,
                                      uint64_t& joins, uint64_t& nodes) {
  if constexpr (L == 3) {
    // each half with candidates (children of members below 64 have no high half)
    const uint64_t cl = Xl & Q.c3l & topl, ch = Xh & Q.c3h & toph;
    if (cl) cq2_push(Q, (cl >> lane) & 1ull, R0 & Xl, 0ull, lane, joins, nodes);
    if (ch) cq2_push(Q, (ch >> lane) & 1ull, R1l & Xl, R1h & Xh, lane, joins, nodes);
  } else {
    uint64_t cl = Xl & readfirstlane64(cm[2 * L]) & topl;
    uint64_t ch = Xh & readfirstlane64(cm[2 * L + 1]) & toph;
    while (cl) {
      const int y = __ffsll((long long)cl) - 1;
      cl &= cl - 1;
      const uint64_t Yl = readlane64(R0, y) & Xl;
      joins += (lane == 0);
      if (__popcll(Yl) >= L - 1) {
        nodes += (lane == 0);
        wdfs2<L - 1>(Q, cm, R0, R1l, R1h, Yl, 0ull, ~0ull, ~0ull, lane, joins, nodes);
      }
    }
    while (ch) {
      const int y = __ffsll((long long)ch) - 1;
      ch &= ch - 1;
      const uint64_t Yl = readlane64(R1l, y) & Xl, Yh = readlane64(R1h, y) & Xh;
      joins += (lane == 0);
      if (__popcll(Yl) + __popcll(Yh) >= L - 1) {
        nodes += (lane == 0);
        wdfs2<L - 1>(Q, cm, R0, R1l, R1h, Yl, Yh, ~0ull, ~0ull, lane, joins, nodes);
      }
    }
  }
}

// Node of level l (4 <= l <= KC_QMAX) whose set C (lane-split `cw`) has 65 to
// 128 members, counted; candidates dealt to `nparts` waves.  `ureg` is the
// wave's evaluation region (16-byte aligned).  It has a single call site (a
// child of a wide node) and unrolls levels 4 and 5 only: every further
// inlined copy of the unrolled levels adds to the register footprint of the
// whole listing kernel.
template <int W, int SP>
__device__ __forceinline__ uint64_t compressed_eval2(const uint32_t* __restrict__ Bl,
                                                     const uint32_t* __restrict__ col, int s, int l, uint32_t cw,
                                                     int lane, uint32_t* __restrict__ ureg, uint64_t& joins,
                                                     uint64_t& nodes, int part, int nparts) {
  uint32_t* rows = ureg;                         // [128][4]
  uint64_t* q = (uint64_t*)(ureg + 512);         // [128][2]
  uint64_t* cm = (uint64_t*)(ureg + 1024);       // [KC_CMAX+1][2]
  uint16_t* mlist = (uint16_t*)(ureg + 1072);    // [128]
  const int hiw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
  if (hiw < 0) return 0;
  const int end = (hiw + 1) * 32 < s ? (hiw + 1) * 32 : s;
  int m = 0;
  for (int p0 = 0; p0 < end; p0 += 64) {
    const int p = p0 + lane;
    const uint32_t word = (uint32_t)__shfl((int)cw, (p >> 5) & 63, 64);
    const bool mem = p < end && ((word >> (p & 31)) & 1u);
    const uint64_t mk = kc_ballot(mem);
    if (mem) mlist[m + kc_mbcnt(mk)] = (uint16_t)p;
    m += __popcll(mk);
  }
  kc_wave_lds_sync();
  const bool valid0 = lane < m, valid1 = lane + 64 < m;
  const int v0 = valid0 ? mlist[lane] : 0, v1 = valid1 ? mlist[lane + 64] : 0;
  // rows: member i = lane gets R0 (members below 64), member 64+lane gets (R1l, R1h)
  uint64_t R0 = 0, R1l = 0, R1h = 0;
  {
    int curw = -1;
    uint32_t b0 = 0, b1 = 0;
    const int m0 = m < 64 ? m : 64;
    for (int jj = 0; jj < m0; ++jj) {
      const int p = __builtin_amdgcn_readlane(v0, jj);
      const int wd = p >> 5;
      if (wd != curw) {
        curw = wd;
        b0 = valid0 ? Bl[wd * SP + v0] : 0u;
        b1 = valid1 ? Bl[wd * SP + v1] : 0u;
      }
      R0 |= (uint64_t)((b0 >> (p & 31)) & 1u) << jj;
      R1l |= (uint64_t)((b1 >> (p & 31)) & 1u) << jj;
    }
    for (int jj = 64; jj < m; ++jj) {
      const int p = __builtin_amdgcn_readlane(v1, jj - 64);
      const int wd = p >> 5;
      if (wd != curw) {
        curw = wd;
        b1 = valid1 ? Bl[wd * SP + v1] : 0u;
      }
      R1h |= (uint64_t)((b1 >> (p & 31)) & 1u) << (jj - 64);
    }
  }
  *(uint2*)(rows + 4 * lane) = make_uint2((uint32_t)R0, (uint32_t)(R0 >> 32));
  *(uint2*)(rows + 4 * lane + 2) = make_uint2(0u, 0u);
  *(uint4*)(rows + 4 * (lane + 64)) =
      make_uint4((uint32_t)R1l, (uint32_t)(R1l >> 32), (uint32_t)R1h, (uint32_t)(R1h >> 32));
  const int c0 = valid0 ? (int)col[v0] : 0, c1 = valid1 ? (int)col[v1] : 0;
#pragma unroll
  for (int c = 0; c <= KC_CMAX; ++c) {
    const uint64_t bl = kc_ballot(valid0 && c0 >= c), bh = kc_ballot(valid1 && c1 >= c);
    if (lane == 0) {
      cm[2 * c] = bl;
      cm[2 * c + 1] = bh;
    }
  }
  CQueue2 Q;
  Q.rows = rows;
  Q.q = q;
  Q.n = 0;
  Q.c2l = kc_ballot(valid0 && c0 >= 2);
  Q.c2h = kc_ballot(valid1 && c1 >= 2);
  Q.c3l = kc_ballot(valid0 && c0 >= 3);
  Q.c3h = kc_ballot(valid1 && c1 >= 3);
  Q.acc = 0;
  const uint64_t Xl = kc_ballot(valid0), Xh = kc_ballot(valid1);
  uint64_t deal = 0;
  for (int j = part; j < 64; j += nparts) deal |= 1ull << j;
  // member 64+i is dealt like member i when nparts divides 64 (1, 4 or 8)
  kc_wave_lds_sync();
#define KC_WD2(LL) \
  case LL: wdfs2<LL>(Q, cm, R0, R1l, R1h, Xl, Xh, deal, deal, lane, joins, nodes); break;
  switch (l) { KC_WD2(4) KC_WD2(5) }
#undef KC_WD2
  if (Q.n > 0) cq2_eval(Q, lane, Q.n, joins);
  kc_wave_lds_sync();
  return Q.acc;
}

// Subtree below candidate j's BitJoin at a node of level l: X2 = R_j.
template <bool PV>
__device__ __forceinline__ uint64_t cdfs_dispatch(int l, const CNode& nd, uint64_t X2, uint64_t& joins,
                                                  uint64_t& nodes, unsigned long long* cnt) {
#define KC_CD(L) \
  case L: return cdfs<PV, L>(nd.rows, nd.rins, nd.mlist, nd.cm, X2, joins, nodes, cnt);
  switch (l - 1) {
    KC_CD(2) KC_CD(3) KC_CD(4) KC_CD(5) KC_CD(6) KC_CD(7) KC_CD(8) KC_CD(9)
  }
#undef KC_CD
  return 0;
}

// Node of level l (2 <= l <= KC_CMAX) whose set C (lane-split `cw`) has at
// most 64 members.  Candidates are dealt to the lanes of `nparts` waves
// (this wave is `part`).  Returns this lane's share of the node's leaves.
template <int W, bool PV, int SP>
__device__ __forceinline__ uint64_t compressed_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                                    const uint32_t* __restrict__ col, int s, int l, uint32_t cw,
                                                    int lane, uint16_t* __restrict__ mlist, uint64_t* __restrict__ rows,
                                                    uint64_t* __restrict__ rins, uint64_t& joins, uint64_t& nodes,
                                                    unsigned long long* cnt, int part, int nparts) {
  const int hiw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
  if (hiw < 0) return 0;
  const int end = (hiw + 1) * 32 < s ? (hiw + 1) * 32 : s;
  int m = 0;
  for (int p0 = 0; p0 < end; p0 += 64) {
    const int p = p0 + lane;
    const uint32_t word = (uint32_t)__shfl((int)cw, (p >> 5) & 63, 64);
    const bool mem = p < end && ((word >> (p & 31)) & 1u);
    const uint64_t mk = kc_ballot(mem);
    if (mem) mlist[m + kc_mbcnt(mk)] = (uint16_t)p;
    m += __popcll(mk);
  }
  kc_wave_lds_sync();
  const bool valid = lane < m;
  const int v = valid ? mlist[lane] : 0;
  // rows: lane j tests each member j' against B(member j)
  uint64_t R = 0, Rin = 0;
  {
    int curw = -1;
    uint32_t bw = 0, biw = 0;
    for (int jj = 0; jj < m; ++jj) {
      const int p = __builtin_amdgcn_readlane(v, jj);
      const int wd = p >> 5;
      if (wd != curw) {
        curw = wd;
        bw = valid ? Bl[wd * SP + v] : 0u;
        if (PV) biw = valid ? Bil[wd * SP + v] : 0u;
      }
      R |= (uint64_t)((bw >> (p & 31)) & 1u) << jj;
      if (PV) Rin |= (uint64_t)((biw >> (p & 31)) & 1u) << jj;
    }
  }
  rows[lane] = R;
  if (PV) rins[lane] = Rin;
  const int cv = valid ? (int)col[v] : 0;
  uint64_t* cmw = rows + 192;  // cm[0..KC_CMAX] after rows and rins
#pragma unroll
  for (int c = 0; c <= KC_CMAX; ++c) {
    const uint64_t b = kc_ballot(valid && cv >= c);
    if (lane == 0) cmw[c] = b;
  }
  const uint64_t cm0 = kc_ballot(valid), cm2 = kc_ballot(valid && cv >= 2);
  const uint64_t cml = kc_ballot(valid && cv >= l);
  CNode nd;
  nd.rows = rows;
  nd.rins = rins;
  nd.mlist = mlist;
  nd.cm = cmw;
  kc_wave_lds_sync();
  if (!PV && l >= 4 && l <= KC_QMAX) {
    CQueue Q;
    Q.rows = rows;
    Q.q = rins;  // the in-rows are not used when counting; 128 entries
    Q.n = 0;
    Q.c2 = cm2;
    Q.c3 = kc_ballot(valid && cv >= 3);
    Q.acc = 0;
    // this wave's share of the node's candidates: members j with j % nparts == part
    uint64_t deal = 0;
    for (int j = part; j < 64; j += nparts) deal |= 1ull << j;
#define KC_WD(LL) \
  case LL: wdfs<LL>(Q, cmw, R, cm0, deal, lane, joins, nodes); break;
    switch (l) { KC_WD(4) KC_WD(5) KC_WD(6) KC_WD(7) KC_WD(8) }
#undef KC_WD
    if (Q.n > 0) cq_eval(Q, lane, Q.n, joins);
    kc_wave_lds_sync();
    return Q.acc;
  }
  uint64_t t = 0;
  // this lane's candidate: member `lane` of the node, if dealt to this wave
  const bool mine = valid && ((lane % nparts) == part);
  if (l == 2) {
    if (mine) {
      const uint64_t X = cm0;
      uint32_t out = 0;
      if ((cm2 >> lane) & 1ull) {
        out = (uint32_t)__popcll(R & X);
        joins++;
      }
      t = out;
      if (PV) {
        const uint32_t in = (uint32_t)__popcll(Rin & X);
        if (out + in) atomicAdd(&cnt[v], (unsigned long long)(out + in));
      }
    }
  } else if (mine && ((cml >> lane) & 1ull)) {
    joins++;
    if (__popcll(R) >= l - 1) {
      nodes++;
      t = cdfs_dispatch<PV>(l, nd, R, joins, nodes, cnt);
      if (PV && t) atomicAdd(&cnt[v], (unsigned long long)t);
    }
  }
  kc_wave_lds_sync();
  return t;
}

// Evaluates a node of level L whose set is the lane-split `cw` on one wave
// (or, at the top of a task, `nparts` waves): compressed when it has at most
// 64 members, lane-parallel at levels 2 and 3, otherwise depth-first with an
// explicit LDS stack whose children are evaluated the same way.  Returns this
// lane's share of the node's leaves.
template <int W, bool PV, bool COMP, int SP>
__device__ uint64_t eval_node(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                              const uint32_t* __restrict__ col, const int32_t* __restrict__ firstpos, int s, int L,
                              uint32_t cw, int lane, uint32_t* __restrict__ stk, int32_t* __restrict__ cur,
                              int32_t* __restrict__ chosen, unsigned long long* __restrict__ tot,
                              uint16_t* __restrict__ mlist, uint64_t* __restrict__ rows, uint64_t* __restrict__ rins,
                              uint16_t* __restrict__ vlist, uint64_t& joins, uint64_t& nodes, uint64_t& wjoins,
                              uint64_t& cjoins, unsigned long long* cnt, int part, int nparts, int cmax, int clev,
                              int32_t* __restrict__ shared_next, uint32_t* __restrict__ ureg) {
  constexpr bool C2 = COMP && !PV && W >= 4 && W <= 16;
  const uint32_t m = split_popc(cw);
  if (COMP && (int)m <= cmax && (int)m <= 64 && L <= KC_CMAX && L >= clev) {
    const uint64_t j0 = joins;
    const uint64_t t = compressed_eval<W, PV, SP>(Bl, Bil, col, s, L, cw, lane, mlist, rows, rins, joins, nodes, cnt,
                                              part, nparts);
    cjoins += joins - j0;
    return t;
  }
  if (L == 2) {
    uint64_t j = 0;
    uint64_t t2 = leaf_eval<W, PV, SP>(Bl, Bil, s, firstpos[2], cw, lane, j, cnt, part, nparts);
    joins += (lane == 0) ? j : 0;
    return (lane == 0) ? t2 : 0;
  }
  if (L == 3)
    return level3_eval<W, PV, SP>(Bl, Bil, s, firstpos[2], firstpos[3], cw, lane, vlist, joins, nodes, cnt, part, nparts);
  // depth-first.  With several waves on the node (nparts > 1) the top-level
  // candidates are taken from a shared counter, one at a time and from the
  // highest position down (those carry the most work), so that the waves
  // balance themselves.
  if (lane < W) stk[lane] = cw;
  if (lane == 0) {
    cur[0] = firstpos[L];
    tot[0] = 0;
  }
  kc_wave_lds_sync();
  uint64_t lane_acc = 0;
  int d = 0;
  int limit = 0;
  if (nparts > 1) {
    const int hw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
    if (hw >= 0) limit = hw * 32 + 32 - __clz((int)kc_readlane(cw, hw));
  }
  for (;;) {
    const int l = L - d;
    const uint32_t mw = lane < W ? stk[d * W + lane] : 0u;
    int x;
    if (d == 0 && nparts > 1) {
      x = -1;
      if (lane == 0) {
        for (;;) {
          // heaviest first: higher positions have more lower-colored neighbours
          const int p = limit - 1 - atomicAdd(shared_next, 1);
          if (p < firstpos[L]) break;
          if ((stk[p >> 5] >> (p & 31)) & 1u) { x = p; break; }
        }
      }
      x = __shfl(x, 0, 64);
    } else {
      const int from = cur[d];
      x = split_next<W>(mw, from, lane);
    }
    if (x < 0) {
      if (d == 0) break;
      if (PV && lane == 0) {
        unsigned long long T = tot[d];
        tot[d - 1] += T;
        if (T) atomicAdd(&cnt[chosen[d - 1]], T);
      }
      kc_wave_lds_sync();
      d--;
      continue;
    }
    if (lane == 0) cur[d] = x + 1;
    kc_wave_lds_sync();
    const uint32_t nw = lane < W ? (Bl[lane * SP + x] & mw) : 0u;
    joins += (lane == 0);
    wjoins += (lane == 0);
    const uint32_t npc = split_popc(nw);
    if ((int)npc < l - 1) continue;
    nodes += (lane == 0);
    const int lc = l - 1;
    const bool comp = COMP && (int)npc <= cmax && (int)npc <= 64 && lc <= KC_CMAX && lc >= clev;
    const bool comp2 = C2 && !comp && (int)npc <= cmax && lc <= KC_Q2MAX && lc >= clev && lc >= 4;
    if (comp || comp2 || lc <= 3) {
      uint64_t tc;
      if (COMP && comp) {
        const uint64_t j0 = joins;
        tc = compressed_eval<W, PV, SP>(Bl, Bil, col, s, lc, nw, lane, mlist, rows, rins, joins, nodes, cnt, 0, 1);
        cjoins += joins - j0;
      } else if (C2 && comp2) {
        const uint64_t j0 = joins;
        tc = compressed_eval2<W, SP>(Bl, col, s, lc, nw, lane, ureg, joins, nodes, 0, 1);
        cjoins += joins - j0;
      } else if (lc == 3)
        tc = level3_eval<W, PV, SP>(Bl, Bil, s, firstpos[2], firstpos[3], nw, lane, vlist, joins, nodes, cnt, 0, 1);
      else {
        uint64_t j = 0;
        uint64_t t2 = leaf_eval<W, PV, SP>(Bl, Bil, s, firstpos[2], nw, lane, j, cnt, 0, 1);
        joins += (lane == 0) ? j : 0;
        tc = (lane == 0) ? t2 : 0;
      }
      lane_acc += tc;
      if (PV) {
        const uint64_t T = kc_wave_sum_u64(tc);
        if (lane == 0) {
          tot[d] += T;
          if (T) atomicAdd(&cnt[x], (unsigned long long)T);
        }
        kc_wave_lds_sync();
      }
    } else {
      if (lane == 0) {
        chosen[d] = x;
        cur[d + 1] = firstpos[lc];
        tot[d + 1] = 0;
      }
      if (lane < W) stk[(d + 1) * W + lane] = nw;
      kc_wave_lds_sync();
      d++;
    }
  }
  return lane_acc;
}

template <int W, int NW, bool PV, bool COMP, bool GB>
// At least 4 waves per SIMD when the bitmaps sit in LDS: the register budget
// stays at 128 VGPRs.  The device-memory layout (GB) serves the widest
// classes, whose lane arrays of W words need more registers.
__global__ __launch_bounds__(64 * NW, GB ? 1 : 4) void k_bitcol_list(ListArgs a) {
  using LY = ListLayout<W, NW, PV, COMP, GB>;
  const int K = a.k + 1;
  constexpr int S = LY::S;
  constexpr int SP = LY::SP;
  extern __shared__ uint32_t lds[];
  const uint32_t* Bl = lds + LY::oB;
  const uint32_t* Bil = lds + LY::oBin;
  uint32_t* col = lds + LY::oCol;
  int32_t* firstpos = (int32_t*)(lds + LY::oFirst);
  uint32_t* C0 = lds + LY::oC0;
  int32_t* sh = (int32_t*)(lds + LY::oSh);  // [0] task lo, [1] task hi
  unsigned long long* shtot = (unsigned long long*)(lds + LY::oSh + 8);
  unsigned long long* cnt = (unsigned long long*)(lds + LY::oCnt(K));

  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  uint32_t* wblk = lds + LY::oWave + wid * LY::wave_words(K);
  unsigned long long* tot = (unsigned long long*)wblk;
  int32_t* cur = (int32_t*)(wblk + 2 * K);
  int32_t* chosen = cur + K;
  uint32_t* stk = (uint32_t*)(chosen + K);
  uint32_t* ureg = wblk + LY::oU(K);
  uint16_t* vlist = (uint16_t*)ureg;
  uint64_t* rows = (uint64_t*)ureg;  // rows[64] | rins or queue[128] | cm[12] | mlist[64] u16
  uint64_t* rins = rows + 64;
  uint16_t* mlist = (uint16_t*)(rows + 204);

  uint64_t my_nodes = 0, my_isect = 0;  // per lane, this task
  uint64_t my_wide = 0, my_comp = 0;    // of which: wave-wide joins, joins on re-encoded 64-bit rows
  // this launch's totals (per lane; the count on thread 0), added to the
  // device counters once at the end: per-task atomics on a handful of
  // addresses serialise when the tasks are many and small
  uint64_t run_nodes = 0, run_isect = 0, run_wide = 0, run_comp = 0, run_work = 0, run_count = 0;
  bool run_ovf = false;

  for (;;) {
    if (tid == 0) {
      unsigned long long t = atomicAdd(a.head, (unsigned long long)a.chunk);
      sh[0] = (int32_t)(t < (unsigned long long)a.ntasks ? t : a.ntasks);
      long long e = (long long)t + a.chunk;
      sh[1] = (int32_t)(e < a.ntasks ? e : a.ntasks);
    }
    __syncthreads();
    const int32_t t_lo = sh[0], t_hi = sh[1];
    __syncthreads();
    if (t_lo >= t_hi) break;
    for (int32_t ti = t_lo; ti < t_hi; ++ti) {
      const uint64_t task = a.tasks[ti];
      const int32_t r = (int32_t)(task >> 32);
      const int v1 = (int)((task >> 16) & 0xffff) - 1;
      const int v2 = (int)(task & 0xffff) - 1;
      const int32_t s = a.ri.s[r];
      const int Wc = d_wclass_words(a.ri.cls[r]);
      const int Sr = 32 * Wc;
      const int64_t bo = a.ri.boff[r], po = a.ri.poff[r];
      const int k = kc_vk(a.vk, a.roots[r], a.k);
      // stage the root's bitmaps into LDS (or read them in place: the
      // classes laid out in device memory have Wc = W, Sr = S)
      if (GB) {
        Bl = a.B + bo;
        if (PV) Bil = a.Bin + bo;
      } else {
        uint32_t* Bw = lds + LY::oB;
        uint32_t* Biw = lds + LY::oBin;
        for (int w = 0; w < W; ++w)
          for (int p = tid; p < S; p += 64 * NW) {
            bool in = w < Wc && p < Sr;
            Bw[w * SP + p] = in ? a.B[bo + (int64_t)w * Sr + p] : 0u;
            if (PV) Biw[w * SP + p] = in ? a.Bin[bo + (int64_t)w * Sr + p] : 0u;
          }
      }
      for (int p = tid; p < S; p += 64 * NW) {
        col[p] = p < s ? (a.noprune ? 0xfffeu : (uint32_t)a.color[po + p]) : 0xffffu;
        if (PV) cnt[p] = 0;
      }
      if (tid == 0) {
        shtot[0] = 0;
        sh[2] = 0;
      }
      __syncthreads();
      // firstpos[c] = number of positions with color < c (colors ascend)
      if (tid <= k + 1 && tid <= KC_KMAX + 1) {
        int lo = 0, hi = s;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if ((int)col[mid] < tid) lo = mid + 1; else hi = mid;
        }
        firstpos[tid] = lo;
      }
      // task node: level L0 and set C0
      int L0 = k - 1;
      if (tid < W) {
        uint32_t c = 0;
        if (tid < Wc) {
          int lo = tid * 32;
          c = lo >= s ? 0u : (s - lo >= 32 ? ~0u : ((1u << (s - lo)) - 1u));
          if (v1 >= 0) c &= Bl[tid * SP + v1];
          if (v2 >= 0) c &= Bl[tid * SP + v2];
        }
        C0[tid] = c;
      }
      if (v1 >= 0) L0--;
      if (v2 >= 0) L0--;
      __syncthreads();
      if (wid == 0) my_nodes += (lane == 0);
      const uint32_t c0w = lane < W ? C0[lane] : 0u;
      const uint64_t wave_total = eval_node<W, PV, COMP, SP>(Bl, Bil, col, firstpos, s, L0, c0w, lane, stk, cur, chosen, tot,
                                                   mlist, rows, rins, vlist, my_isect, my_nodes, my_wide, my_comp, cnt, wid, NW,
                                                   a.cmax, a.clev, &sh[2], ureg);
      {
        const uint64_t wt = kc_wave_sum_u64(wave_total);
        if (lane == 0 && wt) atomicAdd(&shtot[0], (unsigned long long)wt);
      }
      __syncthreads();
      // task epilogue
      const uint64_t T = shtot[0];
      const int32_t u = a.roots[r];
      if (tid == 0 && T) {
        run_ovf |= run_count + T < run_count;
        run_count += T;
        if (a.root_count) kc_add_checked(&a.root_count[u], T, a.flags);
        if (PV) {
          kc_add_checked(&a.pv[u], T, a.flags);
          if (v1 >= 0) kc_add_checked(&a.pv[a.perm[po + v1]], T, a.flags);
          if (v2 >= 0) kc_add_checked(&a.pv[a.perm[po + v2]], T, a.flags);
        }
      }
      if (PV) {
        for (int p = tid; p < s; p += 64 * NW) {
          unsigned long long c = cnt[p];
          if (c) kc_add_checked(&a.pv[a.perm[po + p]], c, a.flags);
        }
      }
      // work counters: the launch's totals, and the per-root log when asked
      {
        const uint64_t ws = (uint64_t)((s + 31) / 32);
        run_nodes += my_nodes;
        run_isect += my_isect;
        run_wide += my_wide;
        run_comp += my_comp;
        run_work += my_isect * ws;
        if (a.root_isect || a.root_work) {
          const uint64_t wi = kc_wave_sum_u64(my_isect);
          if (lane == 0 && wi) {
            if (a.root_isect) atomicAdd((unsigned long long*)&a.root_isect[u], (unsigned long long)wi);
            if (a.root_work) atomicAdd((unsigned long long*)&a.root_work[u], (unsigned long long)(wi * ws));
          }
        }
      }
      my_nodes = 0;
      my_isect = 0;
      my_wide = 0;
      my_comp = 0;
      __syncthreads();
    }
  }
  {
    const uint64_t wn = kc_wave_sum_u64(run_nodes), wi = kc_wave_sum_u64(run_isect);
    const uint64_t ww = kc_wave_sum_u64(run_wide), wc = kc_wave_sum_u64(run_comp), wk = kc_wave_sum_u64(run_work);
    if (lane == 0 && (wi || wn)) {
      atomicAdd(&a.counters[0], (unsigned long long)wn);
      atomicAdd(&a.counters[1], (unsigned long long)wi);
      atomicAdd(&a.counters[2], (unsigned long long)wk);
      atomicAdd(&a.counters[3], (unsigned long long)ww);
      atomicAdd(&a.counters[4], (unsigned long long)wc);
    }
    if (tid == 0) {
      kc_add_checked(a.count, run_count, a.flags);
      if (run_ovf) atomicOr(a.flags, KC_FLAG_OVERFLOW);
    }
  }
}

// ============================================================== host side
template <int W, int NW, bool PV, bool GB>
static size_t list_lds_bytes(const ListArgs& a) {
  return a.cmax > 0 ? ListLayout<W, NW, PV, true, GB>::bytes(a.k + 1) : ListLayout<W, NW, PV, false, GB>::bytes(a.k + 1);
}

static size_t device_max_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return (size_t)v;
}

// A resolved listing launch: kernel instance, grid and LDS size.  Resolving
// sets the kernel's LDS attribute and queries its occupancy, so a captured
// launch sequence makes no such calls while the stream is being captured.
struct ListLaunch {
  const void* fn = nullptr;
  int64_t grid = 0;
  int threads = 0;
  size_t bytes = 0;
};

template <int W, int NW, bool PV, bool GB>
static int resolve_list(const ListArgs& a, ListLaunch* L) {
  const bool comp = a.cmax > 0;
  const size_t bytes = list_lds_bytes<W, NW, PV, GB>(a);
  auto fn = comp ? k_bitcol_list<W, NW, PV, true, GB> : k_bitcol_list<W, NW, PV, false, GB>;
  KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  int per_cu = 0;
  KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * NW, bytes));
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)per_cu * kc_device_cus();
  if (grid > a.ntasks) grid = a.ntasks;
  if (grid < 1) grid = 1;
  L->fn = (const void*)fn;
  L->grid = grid;
  L->threads = 64 * NW;
  L->bytes = bytes;
  return KC_OK;
}

template <int W, bool PV>
static int resolve_list_nw(const ListArgs& a, int nw, ListLaunch* L) {
  // fewer waves per root when the requested shape's LDS does not fit.  The
  // 24- and 32-word classes also run 16 waves per root: their bitmaps take
  // most of a CU's LDS, so one workgroup per CU is all that fits, and 16
  // waves give each SIMD four.
  const size_t lim = device_max_lds();
  if constexpr (W >= 24 && !PV) {
    if (nw >= 16 && list_lds_bytes<W, 16, PV, false>(a) <= lim) return resolve_list<W, 16, PV, false>(a, L);
  }
  if (nw >= 8 && list_lds_bytes<W, 8, PV, false>(a) <= lim) return resolve_list<W, 8, PV, false>(a, L);
  if (nw >= 2 && list_lds_bytes<W, 4, PV, false>(a) <= lim) return resolve_list<W, 4, PV, false>(a, L);
  if (list_lds_bytes<W, 1, PV, false>(a) <= lim) return resolve_list<W, 1, PV, false>(a, L);
  return KC_EUNSUPPORTED;
}

// Classes whose bitmaps stay in device memory: 8 or 1 waves per root.
template <int W, bool PV>
static int resolve_list_nw_dev(const ListArgs& a, int nw, ListLaunch* L) {
  const size_t lim = device_max_lds();
  if (nw >= 2 && list_lds_bytes<W, 8, PV, true>(a) <= lim) return resolve_list<W, 8, PV, true>(a, L);
  if (list_lds_bytes<W, 1, PV, true>(a) <= lim) return resolve_list<W, 1, PV, true>(a, L);
  return KC_EUNSUPPORTED;
}

// The listing launch of the word classes of 24 to 64 words (kc_bitcol_wide.hip).
int kc_resolve_list_wide(const ListArgs& a, int cls, int nw, bool pv, ListLaunch* L);
