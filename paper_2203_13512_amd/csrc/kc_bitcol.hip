// kc_bitcol.hip -- BitCol (Alg. 6, Sec. 7.4) on gfx950.
//
// Two phases.
//
// 1. Staging (one wave per root u with d+_u >= k-1): the local graph G_u is
//    induced by N+(u) (Sec. 7.2).  Its adjacency is built in LDS as a bit
//    matrix by intersecting every N+(v), v in N+(u), with the sorted N+(u)
//    (lanes over the flattened list of all those entries, binary search in
//    LDS).  Vertices are then colored greedily in descending local degree
//    (ties by ascending id) with the smallest free color, 1-based (Sec. 7.1),
//    and renumbered by (color, id), so that "color < c" is a prefix of the
//    positions.  A second intersection pass writes the encoded out-neighbour
//    bitmaps B(v) = {w adjacent to v : color(w) < color(v)} (Sec. 7.3) -- and,
//    for per-vertex counts, the complementary in-neighbour bitmaps -- straight
//    into the renumbered positions.  Bitmaps go to HBM, column-major per root
//    (word i of position p at i*S + p, S = 32*Wc), with the root's color
//    array, its position -> vertex map and its features.
//
// 2. Listing: a persistent kernel takes work items (a root, or a root with
//    one or two chosen first vertices) from a queue.  A workgroup of NW waves
//    copies the root's bitmaps into LDS (row stride S+1 keeps both access
//    patterns bank-conflict free), distributes the children of the item's
//    node over its waves, and each wave runs BitColList depth-first with an
//    explicit LDS stack.  Internal levels handle one candidate at a time
//    (lane i ANDs and counts word i).  The last level (l = 2) is
//    lane-parallel: each lane takes one candidate w and counts
//    popcount(B(w) & C) with v_and/v_bcnt against the candidate set held in
//    scalar registers.  Pruning follows Alg. 6 exactly: candidates of color
//    < l are skipped, and a child is entered only if its set has >= l-1
//    members.
//
// Per-vertex participation (count mode skips all of this): at a level-2 node
// with set C every member y gains popcount(B(y) & C) + popcount(Bin(y) & C)
// (the leaves in which it is the middle or the last vertex), the vertex chosen
// above gains the node's total, and totals of finished subtrees propagate to
// the vertex chosen at each level, so no per-clique work is needed.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "kc_internal.h"

#define KC_NCLASS 8
static const int kWClass[KC_NCLASS] = {1, 2, 4, 8, 12, 16, 24, 32};

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
  return -1;
}
__device__ __forceinline__ int d_wclass_words(int c) {
  const int t[KC_NCLASS] = {1, 2, 4, 8, 12, 16, 24, 32};
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
static size_t stage_lds_bytes(int WM, bool pv) {
  size_t S = 32 * (size_t)WM;
  return 4 * (S + S + 1 + S + S + S + S + WM + 2) + 4 * (size_t)WM * S * (pv ? 2 : 1) + 64;
}

template <bool PV>
__global__ __launch_bounds__(64) void k_bitcol_stage(StageArgs a, const int32_t* __restrict__ list, int32_t nlist,
                                                     int WM) {
  extern __shared__ uint32_t lds[];
  const int S = 32 * WM;
  int32_t* ids = (int32_t*)lds;
  int32_t* off = ids + S;
  int32_t* deg = off + S + 1;
  int32_t* order = deg + S;
  int32_t* color = order + S;
  int32_t* pos = color + S;
  uint32_t* used = (uint32_t*)(pos + S);
  uint32_t* M1 = used + WM + 2;
  uint32_t* M2 = M1 + (size_t)WM * S;
  const int lane = threadIdx.x;

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
    __syncthreads();
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
    __syncthreads();
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
    __syncthreads();
    // local degrees
    for (int i = lane; i < s; i += 64) {
      int d = 0;
      for (int w = 0; w < Wc; ++w) d += __popc(M1[w * S + i]);
      deg[i] = d;
    }
    __syncthreads();
    // coloring order: degree descending, then id (= local index) ascending
    for (int i = lane; i < s; i += 64) {
      int di = deg[i], rk = 0;
      for (int j = 0; j < s; ++j) {
        int dj = deg[j];
        rk += (dj > di) || (dj == di && j < i);
      }
      order[rk] = i;
    }
    __syncthreads();
    // greedy coloring, one vertex at a time
    const int Wu = (s + 1 + 31) / 32;
    int maxc = 0;
    for (int t = 0; t < s; ++t) {
      const int v = order[t];
      for (int w = lane; w < Wu; w += 64) used[w] = 0;
      __syncthreads();
      for (int j = lane; j < s; j += 64) {
        if ((M1[(j >> 5) * S + v] >> (j & 31)) & 1u) {
          int c = color[j];
          if (c > 0) atomicOr(&used[c >> 5], 1u << (c & 31));
        }
      }
      __syncthreads();
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
      __syncthreads();
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
    __syncthreads();
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
    __syncthreads();
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
      atomicAdd(a.stage_bytes, (unsigned long long)(4ull * ((uint64_t)s + (uint64_t)T)));
    }
    __syncthreads();
  }
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
  unsigned long long* count;
  unsigned long long* pv;
  unsigned long long* counters;  // nodes, isect, work
  uint64_t* root_work;
  uint64_t* root_isect;
  int* flags;
};

// LDS layout of a listing workgroup (offsets in 32-bit words, 64-bit
// fields on even offsets):
//   B[W][S+1] | Bin[W][S+1] (per-vertex) | color[S] | firstpos[KMAX+2] |
//   C0[W] | shared scalars[16] | NW wave blocks | cnt[S] u64 (per-vertex)
// A wave block holds tot[KMAX+1] u64 | cur[KMAX+1] | chosen[KMAX+1] |
// stack[(KMAX+1)][W] | candidate lists[2][S] u16 | pairs[2S] u32.
#define KC_KMAX 32

template <int W, int NW, bool PV>
struct ListLayout {
  static constexpr int S = 32 * W;
  static constexpr int SP = S + 1;  // LDS row stride (bank-conflict free)
  static constexpr int a2(int x) { return (x + 1) & ~1; }
  static constexpr int oB = 0;
  static constexpr int oBin = oB + W * SP;
  static constexpr int oCol = oBin + (PV ? W * SP : 0);
  static constexpr int oFirst = oCol + S;
  static constexpr int oC0 = oFirst + KC_KMAX + 2;
  static constexpr int oSh = a2(oC0 + W);
  static constexpr int oWave = oSh + 16;
  static constexpr int PCAP = 2 * S;  // (x, v) pairs buffered per wave
  static constexpr int wave_words = a2(4 * (KC_KMAX + 1) + (KC_KMAX + 1) * W + S / 2 + S / 2 + PCAP);
  static constexpr int oCnt = oWave + NW * wave_words;
  static constexpr int words = oCnt + (PV ? 2 * S : 0);
  static constexpr size_t bytes() { return 4 * (size_t)words; }
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
template <int W, bool PV>
__device__ __forceinline__ uint64_t leaf_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                              int s, int first2, uint32_t cw, int lane, uint64_t& joins,
                                              unsigned long long* cnt, int chunk0 = 0, int chunk_step = 1) {
  constexpr int SP = 32 * W + 1;
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
template <int W, bool PV>
__device__ __forceinline__ uint64_t level3_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                                int s, int first2, int first3, uint32_t cw, int lane,
                                                uint16_t* __restrict__ vlist, uint64_t& joins, uint64_t& nodes,
                                                unsigned long long* cnt, int part, int nparts) {
  constexpr int SP = 32 * W + 1;
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

// Level-4 node with set C (lane-split `cw`), evaluated lane-parallel over
// (x, v) pairs: lanes first take the members x of C with color >= 4, form
// C3 = B(x) & C and count the members v of C3 with color >= 3; the pairs
// (x, v) of the x with |C3| >= 3 are written to an LDS list and then dealt to
// lanes, each forming C2 = B(v) & C3 and, when |C2| >= 2, counting the
// leaves below it as level3_eval does.  Small level-3 nodes thus share
// passes instead of each leaving most lanes idle.  When a batch of x yields
// more pairs than the buffer holds (dense sets), its x are evaluated one by
// one with level3_eval, which is efficient for large sets.
template <int W, bool PV>
__device__ __forceinline__ uint64_t level4_eval(const uint32_t* __restrict__ Bl, const uint32_t* __restrict__ Bil,
                                                int s, int first2, int first3, int first4, uint32_t cw, int lane,
                                                uint16_t* __restrict__ xlist, uint16_t* __restrict__ vlist,
                                                uint32_t* __restrict__ pairs, int pcap, uint64_t& joins,
                                                uint64_t& nodes, unsigned long long* cnt, int part, int nparts) {
  constexpr int SP = 32 * W + 1;
  const int hiw = kc_wave_max_i32((lane < W && cw) ? lane : -1);
  if (hiw < 0) return 0;
  uint32_t c[W];
#pragma unroll
  for (int i = 0; i < W; ++i) c[i] = kc_readlane(cw, i);
  const int end = (hiw + 1) * 32 < s ? (hiw + 1) * 32 : s;
  int mx = 0;
  for (int p0 = first4 & ~63; p0 < end; p0 += 64) {
    const int p = p0 + lane;
    const uint32_t word = (uint32_t)__shfl((int)cw, (p >> 5) & 63, 64);
    const bool mem = p >= first4 && p < end && ((word >> (p & 31)) & 1u);
    const uint64_t mk = kc_ballot(mem);
    if (mem) xlist[mx + kc_mbcnt(mk)] = (uint16_t)p;
    mx += __popcll(mk);
  }
  kc_wave_lds_sync();
  const int f2w = first2 >> 5, f3w = first3 >> 5;
  const uint32_t f2m = (~0u) << (first2 & 31), f3m = (~0u) << (first3 & 31);
  uint64_t total = 0;
  for (int xb = part * 64; xb < mx; xb += 64 * nparts) {
    const int idx = xb + lane;
    const bool valid = idx < mx;
    const int x = valid ? xlist[idx] : 0;
    uint32_t c3[W];
    int p3 = 0, nv = 0;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      c3[i] = (valid && i <= hiw) ? (Bl[i * SP + x] & c[i]) : 0u;
      p3 += __popc(c3[i]);
      const uint32_t mv = i < f3w ? 0u : (i == f3w ? (c3[i] & f3m) : c3[i]);
      nv += __popc(mv);
    }
    joins += valid ? 1 : 0;
    const bool q = valid && p3 >= 3;
    nodes += q ? 1 : 0;
    if (!q) nv = 0;
    // exclusive prefix of nv over the wave
    int incl = nv;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int P = __shfl(incl, 63, 64);
    const int off = incl - nv;
    if (P == 0) continue;
    if (P > pcap) {
      // dense batch: one level-3 node at a time
      uint64_t qm = kc_ballot(q);
      while (qm) {
        const int fl = __ffsll((long long)qm) - 1;
        qm &= qm - 1;
        const int xx = __shfl(x, fl, 64);
        // lane i needs word i of lane fl's C3
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          uint32_t wv = kc_readlane(c3[i], fl);
          if (lane == i) mine = wv;
        }
        uint64_t t3 = level3_eval<W, PV>(Bl, Bil, s, first2, first3, mine, lane, vlist, joins, nodes, cnt, 0, 1);
        total += t3;
        if (PV) {
          uint64_t T3 = kc_wave_sum_u64(t3);
          if (lane == 0 && T3) atomicAdd(&cnt[xx], (unsigned long long)T3);
        }
      }
      continue;
    }
    // write this lane's pairs
    if (q) {
      int j = off;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        uint32_t m = i < f3w ? 0u : (i == f3w ? (c3[i] & f3m) : c3[i]);
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1;
          pairs[j++] = ((uint32_t)x << 16) | (uint32_t)(i * 32 + b);
        }
      }
    }
    kc_wave_lds_sync();
    for (int pb = 0; pb < P; pb += 64) {
      const int pi = pb + lane;
      if (pi >= P) continue;
      const uint32_t pr = pairs[pi];
      const int px = (int)(pr >> 16), v = (int)(pr & 0xffff);
      uint32_t c2[W];
      int pc = 0;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        c2[i] = i <= hiw ? (Bl[i * SP + px] & c[i] & Bl[i * SP + v]) : 0u;
        pc += __popc(c2[i]);
      }
      joins++;
      if (pc < 2) continue;
      nodes++;
      uint32_t leaf = 0;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        uint32_t m = c2[i];
        if (!PV) m = i < f2w ? 0u : (i == f2w ? (m & f2m) : m);
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1;
          const int w = i * 32 + b;
          uint32_t out = 0;
          if (!PV || w >= first2) {
#pragma unroll
            for (int j = 0; j <= i; ++j) out += (uint32_t)__popc(Bl[j * SP + w] & c2[j]);
            joins++;
          }
          leaf += out;
          if (PV) {
            uint32_t in = 0;
#pragma unroll
            for (int j = i; j < W; ++j) in += (uint32_t)__popc(Bil[j * SP + w] & c2[j]);
            if (out + in) atomicAdd(&cnt[w], (unsigned long long)(out + in));
          }
        }
      }
      total += leaf;
      if (PV && leaf) {
        atomicAdd(&cnt[v], (unsigned long long)leaf);
        atomicAdd(&cnt[px], (unsigned long long)leaf);
      }
    }
    kc_wave_lds_sync();
  }
  return total;
}

template <int W, int NW, bool PV>
__global__ __launch_bounds__(64 * NW) void k_bitcol_list(ListArgs a) {
  using LY = ListLayout<W, NW, PV>;
  constexpr int S = LY::S;
  constexpr int SP = LY::SP;
  extern __shared__ uint32_t lds[];
  uint32_t* Bl = lds + LY::oB;
  uint32_t* Bil = lds + LY::oBin;
  uint32_t* col = lds + LY::oCol;
  int32_t* firstpos = (int32_t*)(lds + LY::oFirst);
  uint32_t* C0 = lds + LY::oC0;
  int32_t* sh = (int32_t*)(lds + LY::oSh);  // [0] task lo, [1] task hi, [2] child cursor
  unsigned long long* shtot = (unsigned long long*)(lds + LY::oSh + 8);
  unsigned long long* cnt = (unsigned long long*)(lds + LY::oCnt);

  const int tid = threadIdx.x;
  const int wid = tid >> 6;
  const int lane = tid & 63;
  uint32_t* wblk = lds + LY::oWave + wid * LY::wave_words;
  unsigned long long* tot = (unsigned long long*)wblk;
  int32_t* cur = (int32_t*)(wblk + 2 * (KC_KMAX + 1));
  int32_t* chosen = cur + (KC_KMAX + 1);
  uint32_t* stk = (uint32_t*)(chosen + (KC_KMAX + 1));
  uint16_t* xlist = (uint16_t*)(stk + (KC_KMAX + 1) * W);
  uint16_t* vlist = xlist + S;
  uint32_t* pairs = (uint32_t*)(vlist + S);

  const int k = a.k;
  uint64_t my_nodes = 0, my_isect = 0;  // per lane

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
      // stage the root's bitmaps into LDS
      for (int w = 0; w < W; ++w)
        for (int p = tid; p < S; p += 64 * NW) {
          bool in = w < Wc && p < Sr;
          Bl[w * SP + p] = in ? a.B[bo + (int64_t)w * Sr + p] : 0u;
          if (PV) Bil[w * SP + p] = in ? a.Bin[bo + (int64_t)w * Sr + p] : 0u;
        }
      for (int p = tid; p < S; p += 64 * NW) {
        col[p] = p < s ? (uint32_t)a.color[po + p] : 0xffffu;
        if (PV) cnt[p] = 0;
      }
      if (tid == 0) {
        sh[2] = 0;
        shtot[0] = 0;
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
      const int first2 = firstpos[2], first3 = firstpos[3];
      if (wid == 0) my_nodes += (lane == 0);
      uint64_t wave_total = 0;  // per lane
      const uint32_t c0w = lane < W ? C0[lane] : 0u;
      if (L0 == 2) {
        // the task node is a level-2 node: its 64-position chunks are dealt
        // round-robin to the waves
        uint64_t j = 0;
        uint64_t t2 = leaf_eval<W, PV>(Bl, Bil, s, first2, c0w, lane, j, cnt, wid, NW);
        wave_total += (lane == 0) ? t2 : 0;
        my_isect += (lane == 0) ? j : 0;
      } else if (L0 == 3) {
        wave_total += level3_eval<W, PV>(Bl, Bil, s, first2, first3, c0w, lane, vlist, my_isect, my_nodes, cnt, wid,
                                         NW);
      } else if (L0 == 4) {
        wave_total += level4_eval<W, PV>(Bl, Bil, s, first2, first3, firstpos[4], c0w, lane, xlist, vlist, pairs,
                                         LY::PCAP, my_isect, my_nodes, cnt, wid, NW);
      } else {
        // children of the task node are handed out to waves
        int limit = 0;
        {
          int hiw = kc_wave_max_i32((lane < W && c0w) ? lane : -1);
          if (hiw >= 0) limit = hiw * 32 + 32 - __clz((int)kc_readlane(c0w, hiw));
        }
        for (;;) {
          int v = -1;
          if (lane == 0) {
            for (;;) {
              int p = atomicAdd(&sh[2], 1) + firstpos[L0];
              if (p >= limit) { v = -1; break; }
              if ((C0[p >> 5] >> (p & 31)) & 1u) { v = p; break; }
            }
          }
          v = __shfl(v, 0, 64);
          if (v < 0) break;
          // BitJoin at the task level
          const uint32_t cw = lane < W ? (Bl[lane * SP + v] & c0w) : 0u;
          my_isect += (lane == 0);
          const uint32_t pc = split_popc(cw);
          if ((int)pc < L0 - 1) continue;
          my_nodes += (lane == 0);
          uint64_t sub = 0;  // per lane share of the child's leaves
          if (L0 - 1 == 4) {
            sub = level4_eval<W, PV>(Bl, Bil, s, first2, first3, firstpos[4], cw, lane, xlist, vlist, pairs, LY::PCAP,
                                     my_isect, my_nodes, cnt, 0, 1);
          } else {
            // depth-first from (L0-1, cw); nodes of level 4 are evaluated whole
            if (lane < W) stk[lane] = cw;
            int d = 0;
            if (lane == 0) { cur[0] = firstpos[L0 - 1]; tot[0] = 0; }
            kc_wave_lds_sync();
            uint64_t lane_acc = 0;  // this lane's leaves below the child, credited per level
            for (;;) {
              const int l = L0 - 1 - d;
              const uint32_t mw = lane < W ? stk[d * W + lane] : 0u;
              const int from = cur[d];
              const int x = split_next<W>(mw, from, lane);
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
              my_isect += (lane == 0);
              const uint32_t npc = split_popc(nw);
              if ((int)npc < l - 1) continue;
              my_nodes += (lane == 0);
              if (l - 1 == 4) {
                uint64_t t3 = level4_eval<W, PV>(Bl, Bil, s, first2, first3, firstpos[4], nw, lane, xlist, vlist,
                                                 pairs, LY::PCAP, my_isect, my_nodes, cnt, 0, 1);
                lane_acc += t3;
                if (PV) {
                  // the node total is needed for the chosen vertices above
                  uint64_t T3 = kc_wave_sum_u64(t3);
                  if (lane == 0) {
                    tot[d] += T3;
                    if (T3) atomicAdd(&cnt[x], (unsigned long long)T3);
                  }
                  kc_wave_lds_sync();
                }
              } else {
                if (lane == 0) {
                  chosen[d] = x;
                  cur[d + 1] = firstpos[l - 1];
                  tot[d + 1] = 0;
                }
                if (lane < W) stk[(d + 1) * W + lane] = nw;
                kc_wave_lds_sync();
                d++;
              }
            }
            sub = lane_acc;
          }
          if (PV) {
            uint64_t T = kc_wave_sum_u64(sub);
            if (lane == 0 && T) atomicAdd(&cnt[v], (unsigned long long)T);
          }
          wave_total += sub;
        }
      }
      {
        const uint64_t wt = kc_wave_sum_u64(wave_total);
        if (lane == 0 && wt) atomicAdd(&shtot[0], (unsigned long long)wt);
      }
      __syncthreads();
      // task epilogue
      const uint64_t T = shtot[0];
      const int32_t u = a.roots[r];
      if (tid == 0 && T) {
        kc_add_checked(a.count, T, a.flags);
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
      // per-root work log (flushed per task)
      {
        const uint64_t wi = kc_wave_sum_u64(my_isect), wn = kc_wave_sum_u64(my_nodes);
        if (lane == 0 && (wi || wn)) {
          if (a.root_isect) atomicAdd((unsigned long long*)&a.root_isect[u], (unsigned long long)wi);
          if (a.root_work)
            atomicAdd((unsigned long long*)&a.root_work[u], (unsigned long long)wi * (uint64_t)((s + 31) / 32));
          atomicAdd(&a.counters[0], (unsigned long long)wn);
          atomicAdd(&a.counters[1], (unsigned long long)wi);
          atomicAdd(&a.counters[2], (unsigned long long)wi * (uint64_t)((s + 31) / 32));
        }
      }
      my_nodes = 0;
      my_isect = 0;
      __syncthreads();
    }
  }
}

// ============================================================== scheduling
__global__ void k_root_sizes(int32_t R, const int32_t* __restrict__ roots, const int32_t* __restrict__ drp,
                             int max_class, int32_t* s_out, int32_t* cls_out, int64_t* bwords, int64_t* pwords,
                             int* flags) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int32_t u = roots[r];
  int32_t s = drp[u + 1] - drp[u];
  int c = d_wclass_of(s);
  if (c < 0 || c > max_class) {
    atomicOr(flags, KC_FLAG_TOOBIG);
    c = 0;
  }
  int W = d_wclass_words(c);
  s_out[r] = s;
  cls_out[r] = c;
  bwords[r] = (int64_t)W * 32 * W;
  pwords[r] = 32 * W;
}

// Work estimate (natural log) of each root under the chosen schedule.
// Degree schedule: log C(d+, k-1), the number of (k-1)-subsets of the root's
// out-neighbours -- a function of d+ alone, so roots are ordered by d+.
// Learned schedule: the MLP's prediction of log(1 + words) from the root's
// features (d+, core number, colors of G_u, |E_u|).
__device__ __forceinline__ float log_binom(float n, float k) {
  if (k > n) return -1.0f;
  return lgammaf(n + 1.0f) - lgammaf(k + 1.0f) - lgammaf(n - k + 1.0f);
}

#define KC_LOGW_BINS 512
#define KC_LOGW_SCALE 8.0f

__global__ void k_sched_logw(int32_t R, int k, const int32_t* __restrict__ s, const float* __restrict__ pred,
                             float* logw, int32_t* hist) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  float lw = pred ? pred[r] : log_binom((float)s[r], (float)(k - 1));
  if (!(lw > -1e30f)) lw = 0.f;  // NaN guard
  logw[r] = lw;
  int b = (int)(lw * KC_LOGW_SCALE);
  b = b < 0 ? 0 : (b >= KC_LOGW_BINS ? KC_LOGW_BINS - 1 : b);
  atomicAdd(&hist[b], 1);
}

// depth 2 above `hi`, depth 1 above `lo` (bin units); a split must leave a
// node of level >= 2 below it.
__global__ void k_sched_depth(int32_t R, int k, const float* __restrict__ logw, int lo_bin, int hi_bin, int force,
                              int32_t* depth) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int b = (int)(logw[r] * KC_LOGW_SCALE);
  int d = 0;
  if (force >= 0) {
    if (b >= lo_bin) d = 1;
    if (b >= hi_bin) d = 2;
    if (force > 0 && d > 0) d = force;
  }
  if (d >= 1 && k < 4) d = 0;
  if (d == 2 && k < 5) d = 1;
  depth[r] = d;
}

// Split generator: one wave per root of depth >= 1.  Performs the BitJoins
// above the split exactly as BitColList would (same pruning), records their
// work, and emits one task per surviving node.  Mode 0 counts tasks, mode 1
// writes them.
struct SplitArgs {
  const int32_t* roots;
  RootInfo ri;
  const uint32_t* B;
  const uint16_t* color;
  const int32_t* depth;
  const float* logw;
  int k;
  uint64_t* tasks;
  int32_t* task_bin;
  unsigned long long* ntasks;
  uint64_t* root_isect;
  uint64_t* root_work;
  unsigned long long* counters;
};

__global__ __launch_bounds__(64) void k_bitcol_split(SplitArgs a, const int32_t* __restrict__ list, int32_t nlist,
                                                     int mode) {
  const int lane = threadIdx.x;
  for (int32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int32_t r = list[li];
    const int dep = a.depth[r];
    const int32_t s = a.ri.s[r];
    const int c = a.ri.cls[r];
    const int Wc = d_wclass_words(c);
    const int Sr = 32 * Wc;
    const uint32_t* Br = a.B + a.ri.boff[r];
    const uint16_t* colr = a.color + a.ri.poff[r];
    const int k = a.k;
    uint64_t nodes = 1, isect = 0;  // the top call
    for (int p0 = 0; p0 < s; p0 += 64) {
      const int v1 = p0 + lane;
      bool ok1 = v1 < s && (int)colr[v1] >= k - 1;
      int pc1 = 0;
      if (ok1)
        for (int w = 0; w < Wc; ++w) pc1 += __popc(Br[w * Sr + v1]);
      isect += (uint64_t)__popcll(kc_ballot(ok1));
      bool child1 = ok1 && pc1 >= k - 2;
      if (dep == 1) {
        uint64_t m = kc_ballot(child1);
        if (m) {
          unsigned long long base = 0;
          if (lane == 0) base = atomicAdd(a.ntasks, (unsigned long long)__popcll(m));
          base = (unsigned long long)__shfl((long long)base, 0, 64);
          if (mode == 1 && child1) {
            unsigned long long o = base + (unsigned long long)kc_mbcnt(m);
            a.tasks[o] = ((uint64_t)(uint32_t)r << 32) | ((uint64_t)(v1 + 1) << 16);
            // sub-task estimate: the root's share in proportion to C(|C1|, k-2)
            float lw = log_binom((float)pc1, (float)(k - 2)) - log_binom((float)s, (float)(k - 1)) + a.logw[r];
            a.task_bin[o] = c * 64 + 63 - kc_key_q(lw);
          }
        }
      } else {
        // depth 2: visit each surviving v1 in turn; lanes over v2
        uint64_t m1 = kc_ballot(child1);
        while (m1) {
          int fl = __ffsll((long long)m1) - 1;
          m1 &= m1 - 1;
          const int x1 = p0 + fl;
          nodes += 1;  // node (k-2, C1)
          uint32_t c1[32];
          for (int w = 0; w < Wc; ++w) c1[w] = Br[w * Sr + x1];
          for (int q0 = 0; q0 < s; q0 += 64) {
            const int v2 = q0 + lane;
            bool mem = v2 < s && ((c1[(v2 >> 5) & 31] >> (v2 & 31)) & 1u);
            bool ok2 = mem && (int)colr[v2] >= k - 2;
            int pc2 = 0;
            if (ok2)
              for (int w = 0; w < Wc; ++w) pc2 += __popc(Br[w * Sr + v2] & c1[w]);
            isect += (uint64_t)__popcll(kc_ballot(ok2));
            bool child2 = ok2 && pc2 >= k - 3;
            uint64_t m = kc_ballot(child2);
            if (m) {
              unsigned long long base = 0;
              if (lane == 0) base = atomicAdd(a.ntasks, (unsigned long long)__popcll(m));
              base = (unsigned long long)__shfl((long long)base, 0, 64);
              if (mode == 1 && child2) {
                unsigned long long o = base + (unsigned long long)kc_mbcnt(m);
                a.tasks[o] = ((uint64_t)(uint32_t)r << 32) | ((uint64_t)(x1 + 1) << 16) | (uint64_t)(v2 + 1);
                float lw = log_binom((float)pc2, (float)(k - 3)) - log_binom((float)s, (float)(k - 1)) + a.logw[r];
                a.task_bin[o] = c * 64 + 63 - kc_key_q(lw);
              }
            }
          }
        }
      }
    }
    if (mode == 1 && lane == 0) {
      const int32_t u = a.roots[r];
      const uint64_t words = isect * (uint64_t)((s + 31) / 32);
      if (a.root_isect) atomicAdd((unsigned long long*)&a.root_isect[u], (unsigned long long)isect);
      if (a.root_work) atomicAdd((unsigned long long*)&a.root_work[u], (unsigned long long)words);
      atomicAdd(&a.counters[0], (unsigned long long)nodes);
      atomicAdd(&a.counters[1], (unsigned long long)isect);
      atomicAdd(&a.counters[2], (unsigned long long)words);
    }
  }
}

__global__ void k_plain_tasks(int32_t R, const int32_t* __restrict__ depth, const int32_t* __restrict__ cls,
                              const float* __restrict__ logw, uint64_t* tasks, int32_t* task_bin,
                              unsigned long long* ntasks) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  bool take = r < R && depth[r] == 0;
  uint64_t m = kc_ballot(take);
  unsigned long long base = 0;
  if (kc_lane() == 0 && m) base = atomicAdd(ntasks, (unsigned long long)__popcll(m));
  base = (unsigned long long)__shfl((long long)base, 0, 64);
  if (take) {
    unsigned long long o = base + (unsigned long long)kc_mbcnt(m);
    tasks[o] = (uint64_t)(uint32_t)r << 32;
    task_bin[o] = cls[r] * 64 + 63 - kc_key_q(logw[r]);
  }
}

__global__ void k_gather_tasks(const uint64_t* __restrict__ in, const int32_t* __restrict__ order, int32_t n,
                               uint64_t* out) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[order[i]];
}

__global__ void k_list_of_depth(int32_t R, const int32_t* __restrict__ depth, int32_t* out, int32_t* nout) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  bool take = r < R && depth[r] > 0;
  uint64_t m = kc_ballot(take);
  int base = 0;
  if (kc_lane() == 0 && m) base = atomicAdd(nout, __popcll(m));
  base = __shfl(base, 0, 64);
  if (take) out[base + kc_mbcnt(m)] = r;
}

// log1p-normalised features for the MLP: x = (log1p(f) - mean) / std.
__global__ void k_mlp_features(int32_t R, const float* __restrict__ f, const float* __restrict__ norm, float* x) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * 4) return;
  int j = i & 3;
  x[i] = (log1pf(f[i]) - norm[j]) / norm[4 + j];
}

__global__ void k_scatter_features(int32_t R, const int32_t* __restrict__ roots, const float* __restrict__ f,
                                   float* out) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * 4) return;
  out[4 * (int64_t)roots[i >> 2] + (i & 3)] = f[i];
}

__global__ void k_add_counters(const unsigned long long* __restrict__ per_class, int ncls, unsigned long long* total) {
  int i = threadIdx.x;
  if (i < 3) {
    unsigned long long t = 0;
    for (int c = 0; c < ncls; ++c) t += per_class[3 * c + i];
    total[i] += t;
  }
}

// ============================================================== host side
template <int W, int NW, bool PV>
static int launch_list(const ListArgs& a, hipStream_t st) {
  using LY = ListLayout<W, NW, PV>;
  const size_t bytes = LY::bytes();
  auto fn = k_bitcol_list<W, NW, PV>;
  KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  int per_cu = 0;
  KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * NW, bytes));
  if (per_cu < 1) per_cu = 1;
  int64_t grid = (int64_t)per_cu * kc_device_cus();
  if (grid > a.ntasks) grid = a.ntasks;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64 * NW), bytes, st, a);
  KC_HIP(hipGetLastError());
  return KC_OK;
}

template <int W, bool PV>
static int launch_list_nw(const ListArgs& a, int nw, hipStream_t st) {
  if (nw >= 4) return launch_list<W, 4, PV>(a, st);
  if (nw == 2) return launch_list<W, 2, PV>(a, st);
  return launch_list<W, 1, PV>(a, st);
}

static int launch_list_class(const ListArgs& a, int cls, int nw, bool pv, hipStream_t st) {
#define KC_CASE(c, W)                                                            \
  case c:                                                                        \
    return pv ? launch_list_nw<W, true>(a, nw, st) : launch_list_nw<W, false>(a, nw, st);
  switch (cls) {
    KC_CASE(0, 1)
    KC_CASE(1, 2)
    KC_CASE(2, 4)
    KC_CASE(3, 8)
    KC_CASE(4, 12)
    KC_CASE(5, 16)
    case 6:
      if (pv) return KC_EUNSUPPORTED;
      return launch_list_nw<24, false>(a, nw, st);
    case 7:
      if (pv) return KC_EUNSUPPORTED;
      return launch_list_nw<32, false>(a, nw, st);
  }
#undef KC_CASE
  return KC_EUNSUPPORTED;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  int init() {
    KC_HIP(hipEventCreate(&a));
    KC_HIP(hipEventCreate(&b));
    return KC_OK;
  }
  float ms() {
    float t = 0.f;
    if (hipEventSynchronize(b) != hipSuccess) return 0.f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return 0.f;
    return t;
  }
};

int kc_list_bitcol(kc_list_ctx& c, kc_scratch& scr, hipStream_t st) {
  const int32_t R = c.nroots;
  if (R == 0) return KC_OK;
  const bool pv = c.pv != nullptr;
  const kc_options* opt = c.opt;
  const int max_class = pv ? 5 : 7;
  EventPair ev_stage, ev_sched, ev_list;
  KC_TRY(ev_stage.init());
  KC_TRY(ev_sched.init());
  KC_TRY(ev_list.init());
  KC_HIP(hipEventRecord(ev_stage.a, st));

  RootInfo ri;
  int64_t *bwords, *pwords;
  KC_TRY(scr.get(&ri.s, R));
  KC_TRY(scr.get(&ri.cls, R));
  KC_TRY(scr.get(&ri.boff, (size_t)R + 1));
  KC_TRY(scr.get(&ri.poff, (size_t)R + 1));
  KC_TRY(scr.get(&bwords, (size_t)R + 1));
  KC_TRY(scr.get(&pwords, (size_t)R + 1));
  k_root_sizes<<<(R + 255) / 256, 256, 0, st>>>(R, c.roots, c.drp, max_class, ri.s, ri.cls, bwords, pwords, c.flags);
  KC_HIP(hipGetLastError());
  int64_t* totals;
  KC_TRY(scr.get(&totals, 4));
  KC_TRY(kc_scan_i64(bwords, ri.boff, R, totals, st));
  KC_TRY(kc_scan_i64(pwords, ri.poff, R, totals + 1, st));
  int64_t htot[2];
  int hflags = 0;
  KC_HIP(hipMemcpyAsync(htot, totals, sizeof(htot), hipMemcpyDeviceToHost, st));
  KC_HIP(hipMemcpyAsync(&hflags, c.flags, sizeof(int), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;

  uint32_t *B, *Bin = nullptr;
  int32_t* perm;
  uint16_t* color;
  float* feat;
  KC_TRY(scr.get(&B, (size_t)htot[0]));
  if (pv) KC_TRY(scr.get(&Bin, (size_t)htot[0]));
  KC_TRY(scr.get(&perm, (size_t)htot[1]));
  KC_TRY(scr.get(&color, (size_t)htot[1]));
  KC_TRY(scr.get(&feat, (size_t)R * 4));

  // ---- staging, one launch per bitmap class
  int32_t* byclass;
  int32_t hoff[KC_NCLASS + 1];
  KC_TRY(scr.get(&byclass, R));
  KC_TRY(kc_bin_sort(ri.cls, R, KC_NCLASS, byclass, hoff, scr, st));
  StageArgs sa;
  sa.drp = c.drp;
  sa.dcol = c.dcol;
  sa.roots = c.roots;
  sa.core = c.core;
  sa.ri = ri;
  sa.B = B;
  sa.Bin = Bin;
  sa.perm = perm;
  sa.color = color;
  sa.features = feat;
  sa.stage_bytes = c.counters + 3;
  sa.flags = c.flags;
  for (int cl = 0; cl < KC_NCLASS; ++cl) {
    int32_t cnt = hoff[cl + 1] - hoff[cl];
    if (cnt <= 0) continue;
    int WM = kWClass[cl];
    size_t bytes = stage_lds_bytes(WM, pv);
    auto fn = pv ? k_bitcol_stage<true> : k_bitcol_stage<false>;
    KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    int per_cu = 0;
    KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, bytes));
    int64_t grid = (int64_t)(per_cu < 1 ? 1 : per_cu) * kc_device_cus() * 4;
    if (grid > cnt) grid = cnt;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), bytes, st, sa, byclass + hoff[cl], cnt, WM);
    KC_HIP(hipGetLastError());
  }
  KC_HIP(hipEventRecord(ev_stage.b, st));
  if (c.root_features) {
    k_scatter_features<<<(R * 4 + 255) / 256, 256, 0, st>>>(R, c.roots, feat, c.root_features);
    KC_HIP(hipGetLastError());
  }

  // ---- schedule
  KC_HIP(hipEventRecord(ev_sched.a, st));
  float *pred = nullptr, *logw;
  int32_t* depth;
  KC_TRY(scr.get(&logw, R));
  KC_TRY(scr.get(&depth, R));
  const bool learned = opt && opt->schedule == KC_SCHED_LEARNED;
  if (learned) {
    if (!opt->mlp_params || !opt->mlp_norm) return KC_EINVAL;
    float* x;
    KC_TRY(scr.get(&x, (size_t)R * 4));
    KC_TRY(scr.get(&pred, R));
    k_mlp_features<<<(R * 4 + 255) / 256, 256, 0, st>>>(R, feat, opt->mlp_norm, x);
    KC_HIP(hipGetLastError());
    KC_TRY(kc_mlp_forward_dev(opt->mlp_params, x, R, pred, st));
  }
  int32_t* hist;
  KC_TRY(scr.get(&hist, KC_LOGW_BINS));
  KC_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * KC_LOGW_BINS, st));
  k_sched_logw<<<(R + 255) / 256, 256, 0, st>>>(R, c.k, ri.s, pred, logw, hist);
  KC_HIP(hipGetLastError());
  std::vector<int32_t> hh(KC_LOGW_BINS);
  KC_HIP(hipMemcpyAsync(hh.data(), hist, sizeof(int32_t) * KC_LOGW_BINS, hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  // split thresholds, in histogram bins
  const int slots = kc_device_cus() * 4;
  int lo_bin = KC_LOGW_BINS, hi_bin = KC_LOGW_BINS;
  if (opt && opt->split_threshold > 0.f) {
    lo_bin = (int)(opt->split_threshold * KC_LOGW_SCALE);
    hi_bin = (int)((opt->split_threshold + 4.0f) * KC_LOGW_SCALE);
  } else if (learned) {
    // predicted total work; a root heavier than 1/(8 slots) of it is split
    // once, and one heavier than 64 such shares twice
    double tot = 0.0;
    for (int b = 0; b < KC_LOGW_BINS; ++b) tot += (double)hh[b] * exp((b + 0.5) / KC_LOGW_SCALE);
    double target = tot / (8.0 * slots);
    if (target > 1.0) {
      lo_bin = (int)(log(target) * KC_LOGW_SCALE) + 1;
      hi_bin = (int)(log(target * 64.0) * KC_LOGW_SCALE) + 1;
    }
  } else {
    // degree schedule: the slots/4 roots of largest d+ are split twice, the
    // next 4 x slots once
    const int64_t n2 = slots / 4, n1 = (int64_t)slots * 4;
    int64_t cum = 0;
    for (int b = KC_LOGW_BINS - 1; b >= 0; --b) {
      cum += hh[b];
      if (hi_bin == KC_LOGW_BINS && cum >= n2) hi_bin = b + 1;
      if (cum >= n2 + n1) { lo_bin = b + 1; break; }
    }
    if (lo_bin > hi_bin) lo_bin = hi_bin;
  }
  const int force = opt ? opt->split : 0;
  k_sched_depth<<<(R + 255) / 256, 256, 0, st>>>(R, c.k, logw, lo_bin, hi_bin, force, depth);
  KC_HIP(hipGetLastError());
  // roots to split
  int32_t *splitlist, *nsplit;
  KC_TRY(scr.get(&splitlist, R));
  KC_TRY(scr.get(&nsplit, 2));
  KC_HIP(hipMemsetAsync(nsplit, 0, sizeof(int32_t), st));
  k_list_of_depth<<<(R + 255) / 256, 256, 0, st>>>(R, depth, splitlist, nsplit);
  KC_HIP(hipGetLastError());
  int32_t hns = 0;
  KC_HIP(hipMemcpyAsync(&hns, nsplit, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  SplitArgs sp;
  sp.roots = c.roots;
  sp.ri = ri;
  sp.B = B;
  sp.color = color;
  sp.depth = depth;
  sp.logw = logw;
  sp.k = c.k;
  sp.root_isect = c.root_isect;
  sp.root_work = c.root_work;
  sp.counters = c.counters;
  unsigned long long* ntask_dev;
  KC_TRY(scr.get(&ntask_dev, 2));
  KC_HIP(hipMemsetAsync(ntask_dev, 0, sizeof(unsigned long long), st));
  unsigned long long n_split_tasks = 0;
  if (hns > 0) {
    sp.tasks = nullptr;
    sp.task_bin = nullptr;
    sp.ntasks = ntask_dev;
    k_bitcol_split<<<(unsigned)(hns < 65536 ? hns : 65536), 64, 0, st>>>(sp, splitlist, hns, 0);
    KC_HIP(hipGetLastError());
    KC_HIP(hipMemcpyAsync(&n_split_tasks, ntask_dev, sizeof(n_split_tasks), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
  }
  const int64_t cap = (int64_t)R + (int64_t)n_split_tasks;
  if (cap >= (int64_t)INT32_MAX) return KC_EUNSUPPORTED;
  uint64_t *tasks, *tasks_sorted;
  int32_t *task_bin, *order;
  KC_TRY(scr.get(&tasks, (size_t)cap + 1));
  KC_TRY(scr.get(&tasks_sorted, (size_t)cap + 1));
  KC_TRY(scr.get(&task_bin, (size_t)cap + 1));
  KC_TRY(scr.get(&order, (size_t)cap + 1));
  KC_HIP(hipMemsetAsync(ntask_dev, 0, sizeof(unsigned long long), st));
  k_plain_tasks<<<(R + 255) / 256, 256, 0, st>>>(R, depth, ri.cls, logw, tasks, task_bin, ntask_dev);
  KC_HIP(hipGetLastError());
  if (hns > 0) {
    sp.tasks = tasks;
    sp.task_bin = task_bin;
    sp.ntasks = ntask_dev;
    k_bitcol_split<<<(unsigned)(hns < 65536 ? hns : 65536), 64, 0, st>>>(sp, splitlist, hns, 1);
    KC_HIP(hipGetLastError());
  }
  unsigned long long ntasks_h = 0;
  KC_HIP(hipMemcpyAsync(&ntasks_h, ntask_dev, sizeof(ntasks_h), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int32_t NT = (int32_t)ntasks_h;
  const int NB = KC_NCLASS * 64;
  std::vector<int32_t> boff(NB + 1);
  KC_TRY(kc_bin_sort(task_bin, NT, NB, order, boff.data(), scr, st));
  if (NT > 0) {
    k_gather_tasks<<<(NT + 255) / 256, 256, 0, st>>>(tasks, order, NT, tasks_sorted);
    KC_HIP(hipGetLastError());
  }
  KC_HIP(hipEventRecord(ev_sched.b, st));

  // ---- listing: one persistent launch per bitmap class, heaviest first
  unsigned long long* heads;
  KC_TRY(scr.get(&heads, KC_NCLASS));
  KC_HIP(hipMemsetAsync(heads, 0, sizeof(unsigned long long) * KC_NCLASS, st));
  KC_HIP(hipEventRecord(ev_list.a, st));
  int launches = 0;
  EventPair ev_cls[KC_NCLASS];
  unsigned long long* cls_ctr;
  KC_TRY(scr.get(&cls_ctr, 3 * KC_NCLASS));
  KC_HIP(hipMemsetAsync(cls_ctr, 0, sizeof(unsigned long long) * 3 * KC_NCLASS, st));
  for (int cl = KC_NCLASS - 1; cl >= 0; --cl) {
    int32_t lo = boff[cl * 64], hi = boff[(cl + 1) * 64];
    if (hi <= lo) continue;
    KC_TRY(ev_cls[cl].init());
    KC_HIP(hipEventRecord(ev_cls[cl].a, st));
    ListArgs la;
    la.roots = c.roots;
    la.ri = ri;
    la.B = B;
    la.Bin = Bin;
    la.perm = perm;
    la.color = color;
    la.tasks = tasks_sorted + lo;
    la.ntasks = hi - lo;
    la.head = heads + cl;
    int nw = opt && opt->waves_per_root > 0 ? opt->waves_per_root : (kWClass[cl] >= 8 ? 4 : 1);
    int chunk = opt && opt->chunk > 0 ? opt->chunk : (kWClass[cl] >= 8 ? 1 : 8);
    la.chunk = chunk;
    la.k = c.k;
    la.count = c.count;
    la.pv = c.pv;
    la.counters = cls_ctr + 3 * cl;
    la.root_work = c.root_work;
    la.root_isect = c.root_isect;
    la.flags = c.flags;
    KC_TRY(launch_list_class(la, cl, nw, pv, st));
    KC_HIP(hipEventRecord(ev_cls[cl].b, st));
    launches++;
  }
  k_add_counters<<<1, 64, 0, st>>>(cls_ctr, KC_NCLASS, c.counters);
  KC_HIP(hipGetLastError());
  KC_HIP(hipEventRecord(ev_list.b, st));
  if (c.stats) {
    c.stats->stage_ms += ev_stage.ms();
    c.stats->sched_ms += ev_sched.ms();
    c.stats->list_ms += ev_list.ms();
    c.stats->list_launches += launches;
    c.stats->n_tasks += NT;
    unsigned long long hc[3 * KC_NCLASS];
    KC_HIP(hipMemcpyAsync(hc, cls_ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    for (int cl = 0; cl < KC_NCLASS; ++cl) {
      if (ev_cls[cl].a) c.stats->class_ms[cl] = ev_cls[cl].ms();
      c.stats->class_work[cl] = hc[3 * cl + 2];
      c.stats->class_tasks[cl] = boff[(cl + 1) * 64] - boff[cl * 64];
    }
  }
  return KC_OK;
}
