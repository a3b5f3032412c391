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
#include "kc_bitcol.h"

// ============================================================== listing output
// Emission of every clique (kclique_list): one wave per root, BitColList
// (Alg. 6) depth-first on the root's bitmaps in LDS with the same pruning
// (candidates of color >= l only, a child entered when it has >= l-1
// members).  At l = 2 the node's candidate v and each w of B(v) & C give the
// clique R + {v, w} (the emit step of Alg. 6): the wave reserves one row per
// clique with one atomic, lane i writes the rows of the members in word i.
struct EmitArgs {
  const int32_t* roots;
  RootInfo ri;
  const uint32_t* B;
  const int32_t* perm;
  const uint16_t* color;
  int k;
  const int32_t* vk;
  kc_emit e;
  unsigned long long* count;
  int* flags;
};

template <int W, bool GB>
struct EmitLayout {
  static constexpr int S = 32 * W;
  static constexpr int SP = GB ? S : S + 1;
  static constexpr int oStk = GB ? 0 : W * SP;              // candidate sets, [KMAX][W]
  static constexpr int oGid = oStk + KC_KMAX * W;            // position -> vertex id, [S]
  static constexpr int oFirst = oGid + S;                    // first position of each color, [KMAX+2]
  static constexpr int oChosen = oFirst + KC_KMAX + 2;       // vertex chosen at each level, [KMAX]
  static constexpr int oCur = oChosen + KC_KMAX;             // next position to try, [KMAX]
  static constexpr int words = oCur + KC_KMAX;
};

template <int W, bool GB>
__global__ __launch_bounds__(64) void k_bitcol_emit(EmitArgs a, const int32_t* __restrict__ list, int32_t nlist) {
  using LY = EmitLayout<W, GB>;
  constexpr int S = LY::S, SP = LY::SP;
  extern __shared__ uint32_t lds[];
  const uint32_t* Bl = lds;
  uint32_t* stk = lds + LY::oStk;
  int32_t* gid = (int32_t*)(lds + LY::oGid);
  int32_t* firstpos = (int32_t*)(lds + LY::oFirst);
  int32_t* chosen = (int32_t*)(lds + LY::oChosen);
  int32_t* cur = (int32_t*)(lds + LY::oCur);
  const int lane = threadIdx.x;
  uint64_t found = 0;
  for (int32_t li = blockIdx.x; li < nlist; li += gridDim.x) {
    const int32_t r = list[li];
    const int32_t u = a.roots[r];
    const int32_t s = a.ri.s[r];
    const int Wc = d_wclass_words(a.ri.cls[r]);
    const int Sr = 32 * Wc;
    const int64_t bo = a.ri.boff[r], po = a.ri.poff[r];
    const int k = kc_vk(a.vk, u, a.k);
    if (GB) {
      Bl = a.B + bo;  // the widest classes read the staged block in place (Wc = W)
    } else {
      for (int w = 0; w < W; ++w)
        for (int p = lane; p < S; p += 64) lds[w * SP + p] = (w < Wc && p < Sr) ? a.B[bo + (int64_t)w * Sr + p] : 0u;
    }
    for (int p = lane; p < S; p += 64) gid[p] = p < s ? a.perm[po + p] : -1;
    if (lane <= k + 1 && lane <= KC_KMAX + 1) {
      int lo = 0, hi = s;  // colors ascend with position
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)a.color[po + mid] < lane) lo = mid + 1; else hi = mid;
      }
      firstpos[lane] = lo;
    }
    const int L0 = k - 1;
    if (lane < W) {
      const int lo = lane * 32;
      stk[lane] = lo >= s ? 0u : (s - lo >= 32 ? ~0u : ((1u << (s - lo)) - 1u));
    }
    __syncthreads();
    if (lane == 0) cur[0] = firstpos[L0];
    kc_wave_lds_sync();
    int d = 0;
    for (;;) {
      const int l = L0 - d;
      const uint32_t mw = lane < W ? stk[d * W + lane] : 0u;
      const int x = split_next<W>(mw, cur[d], lane);
      if (x < 0) {
        if (d == 0) break;
        d--;
        continue;
      }
      if (lane == 0) cur[d] = x + 1;
      kc_wave_lds_sync();
      const uint32_t nw = lane < W ? (Bl[lane * SP + x] & mw) : 0u;
      const int pc = __popc(nw);
      if (l == 2) {
        // exclusive prefix of the members over the words, then the rows
        int incl = pc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        const int t = __shfl(incl, 63, 64);
        if (t == 0) continue;
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(a.e.pos, (unsigned long long)t);
        base = (unsigned long long)__shfl((long long)base, 0, 64);
        found += t;
        uint32_t m = nw;
        unsigned long long row = base + (unsigned long long)(incl - pc);
        const int32_t vx = gid[x];
        while (m) {
          const int b = __ffs(m) - 1;
          m &= m - 1;
          if (row < (unsigned long long)a.e.cap) {
            int32_t* o = a.e.out + (int64_t)row * a.k;
            o[0] = u;
            for (int i = 0; i < d; ++i) o[1 + i] = chosen[i];
            o[1 + d] = vx;
            o[2 + d] = gid[lane * 32 + b];
          }
          row++;
        }
      } else if ((int)split_popc(nw) >= l - 1) {
        if (lane == 0) {
          chosen[d] = gid[x];
          cur[d + 1] = firstpos[l - 1];
        }
        if (lane < W) stk[(d + 1) * W + lane] = nw;
        kc_wave_lds_sync();
        d++;
      }
    }
    __syncthreads();
  }
  const uint64_t tot = kc_wave_sum_u64(lane == 0 ? found : 0);
  if (lane == 0 && tot) kc_add_checked(a.count, tot, a.flags);
}

template <int W, bool GB = false>
static int launch_emit(const EmitArgs& a, const int32_t* list, int32_t nlist, hipStream_t st) {
  const size_t bytes = 4 * (size_t)EmitLayout<W, GB>::words;
  auto fn = k_bitcol_emit<W, GB>;
  KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  int per_cu = 0;
  KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, bytes));
  int64_t grid = (int64_t)(per_cu < 1 ? 1 : per_cu) * kc_device_cus() * 2;
  if (grid > nlist) grid = nlist;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), bytes, st, a, list, nlist);
  KC_HIP(hipGetLastError());
  return KC_OK;
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

__global__ void k_sched_logw(int32_t R, int k, const int32_t* __restrict__ roots, const int32_t* vk,
                             const int32_t* __restrict__ s, const int32_t* __restrict__ cls,
                             const float* __restrict__ pred, float* logw, int32_t* hist) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int kr = kc_vk(vk, roots[r], k);
  float lw = pred ? pred[r] : log_binom((float)s[r], (float)(kr - 1));
  if (!(lw > -1e30f)) lw = 0.f;  // NaN guard
  logw[r] = lw;
  int b = (int)(lw * KC_LOGW_SCALE);
  b = b < 0 ? 0 : (b >= KC_LOGW_BINS ? KC_LOGW_BINS - 1 : b);
  atomicAdd(&hist[cls[r] * KC_LOGW_BINS + b], 1);  // one histogram per word class
}

struct ClassBins {
  int lo[KC_NCLASS];
  int hi[KC_NCLASS];
};

// depth 2 above `hi`, depth 1 above `lo` (bin units); a split must leave a
// node of level >= 2 below it.
__global__ void k_sched_depth(int32_t R, int k0, const int32_t* __restrict__ roots, const int32_t* vk,
                              const int32_t* __restrict__ cls, const float* __restrict__ logw, ClassBins cb,
                              int force, int32_t* depth) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int k = kc_vk(vk, roots[r], k0);
  const int lo_bin = cb.lo[cls[r]], hi_bin = cb.hi[cls[r]];
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
  const int32_t* vk;
  int noprune;
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
    const int k = kc_vk(a.vk, a.roots[r], a.k);
    uint64_t nodes = 1, isect = 0;  // the top call
    for (int p0 = 0; p0 < s; p0 += 64) {
      const int v1 = p0 + lane;
      bool ok1 = v1 < s && (a.noprune || (int)colr[v1] >= k - 1);
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
            bool ok2 = mem && (a.noprune || (int)colr[v2] >= k - 2);
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

// per-class counters (KC_NCTR each) into the call's totals: nodes, isect and
// work to slots 0-2, the two join kinds to slots 4-5 (slot 3 is staging)
#define KC_NCTR 5
__global__ void k_add_counters(const unsigned long long* __restrict__ per_class, int ncls, unsigned long long* total) {
  int i = threadIdx.x;
  if (i < KC_NCTR) {
    unsigned long long t = 0;
    for (int c = 0; c < ncls; ++c) t += per_class[KC_NCTR * c + i];
    total[i < 3 ? i : i + 1] += t;
  }
}

static int resolve_list_class(const ListArgs& a, int cls, int nw, bool pv, ListLaunch* L) {
#define KC_CASE(c, W)                                                            \
  case c:                                                                        \
    return pv ? resolve_list_nw<W, true>(a, nw, L) : resolve_list_nw<W, false>(a, nw, L);
  switch (cls) {
    KC_CASE(0, 1)
    KC_CASE(1, 2)
    KC_CASE(2, 4)
    KC_CASE(3, 8)
    KC_CASE(4, 12)
    KC_CASE(5, 16)
    default:
      return kc_resolve_list_wide(a, cls, nw, pv, L);
  }
#undef KC_CASE
}

static int run_list(const ListLaunch& L, const ListArgs& a, hipStream_t st) {
  ListArgs arg = a;
  void* args[] = {(void*)&arg};
  KC_HIP(hipLaunchKernel(L.fn, dim3((unsigned)L.grid), dim3((unsigned)L.threads), args, L.bytes, st));
  return KC_OK;
}

static int launch_list_class(const ListArgs& a, int cls, int nw, bool pv, hipStream_t st) {
  ListLaunch L;
  KC_TRY(resolve_list_class(a, cls, nw, pv, &L));
  return run_list(L, a, st);
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// The listing phase of a prepared call, replayable: the queue heads and the
// per-class counters are cleared by a kernel (not a memset), the classes'
// kernels follow each other on one stream, and the counters are added to the
// call's totals.
struct BitcolReplay {
  ListArgs la[KC_NCLASS];
  ListLaunch ll[KC_NCLASS];
  bool used[KC_NCLASS] = {};
  unsigned long long* heads = nullptr;
  unsigned long long* cls_ctr = nullptr;
  unsigned long long* counters = nullptr;
};

static int bitcol_replay_launch(const void* state, hipStream_t st) {
  const BitcolReplay& R = *(const BitcolReplay*)state;
  k_fill_u64<<<1, 64, 0, st>>>(R.heads, KC_NCLASS, 0ull);
  k_fill_u64<<<1, 64, 0, st>>>(R.cls_ctr, KC_NCTR * KC_NCLASS, 0ull);
  KC_HIP(hipGetLastError());
  for (int cl = KC_NCLASS - 1; cl >= 0; --cl)
    if (R.used[cl]) KC_TRY(run_list(R.ll[cl], R.la[cl], st));
  k_add_counters<<<1, 64, 0, st>>>(R.cls_ctr, KC_NCLASS, R.counters);
  KC_HIP(hipGetLastError());
  return KC_OK;
}

static void bitcol_replay_destroy(void* state) { delete (BitcolReplay*)state; }

// A pair of timing events, created only when statistics are asked for.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  int init(bool on) {
    if (!on) return KC_OK;
    KC_HIP(hipEventCreate(&a));
    KC_HIP(hipEventCreate(&b));
    return KC_OK;
  }
  int start(hipStream_t s) {
    if (a) KC_HIP(hipEventRecord(a, s));
    return KC_OK;
  }
  int stop(hipStream_t s) {
    if (b) KC_HIP(hipEventRecord(b, s));
    return KC_OK;
  }
  float ms() {
    float t = 0.f;
    if (!a || !b) return 0.f;
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
  // The classes whose bitmaps stay in device memory are enabled up to
  // KC_DEVMEM_KMAX only: a run at k = 16 on them faulted the GPU and its cause
  // is not found yet, so larger k is refused (KC_EUNSUPPORTED) rather than run.
  const int max_class = c.k <= KC_DEVMEM_KMAX ? KC_NCLASS - 1 : (pv ? 5 : 7);
  const bool timed = c.stats != nullptr && !c.size_only;
  EventPair ev_stage, ev_sched, ev_list;
  KC_TRY(ev_stage.init(timed));
  KC_TRY(ev_sched.init(timed));
  KC_TRY(ev_list.init(timed));
  KC_TRY(ev_stage.start(st));

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
  KC_TRY(kc_scan_i64(bwords, ri.boff, R, totals, scr, st));
  KC_TRY(kc_scan_i64(pwords, ri.poff, R, totals + 1, scr, st));
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
    const bool in_dev = class_in_device_memory(cl, pv);
    size_t bytes = stage_lds_bytes(WM, pv, !in_dev);
    auto fn = pv ? k_bitcol_stage<true> : k_bitcol_stage<false>;
    KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    int per_cu = 0;
    KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, bytes));
    int64_t grid = (int64_t)(per_cu < 1 ? 1 : per_cu) * kc_device_cus() * 4;
    uint32_t* mat = nullptr;
    if (in_dev) {
      // one adjacency matrix (two with per-vertex output) per workgroup
      if (grid > 256) grid = 256;
      if (grid > cnt) grid = cnt;
      KC_TRY(scr.get(&mat, (size_t)grid * (pv ? 2 : 1) * (size_t)WM * 32 * WM));
    }
    if (grid > cnt) grid = cnt;
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), bytes, st, sa, byclass + hoff[cl], cnt, WM, mat);
    KC_HIP(hipGetLastError());
  }
  KC_TRY(ev_stage.stop(st));
  if (c.emit) {
    // listing output: every root in one launch per word class, no schedule
    EmitArgs ea;
    ea.roots = c.roots;
    ea.ri = ri;
    ea.B = B;
    ea.perm = perm;
    ea.color = color;
    ea.k = c.k;
    ea.vk = c.vk;
    ea.e = *c.emit;
    ea.count = c.count;
    ea.flags = c.flags;
    for (int cl = 0; cl < KC_NCLASS; ++cl) {
      const int32_t cnt = hoff[cl + 1] - hoff[cl];
      if (cnt <= 0 || c.size_only) continue;
      const int32_t* lst = byclass + hoff[cl];
      switch (cl) {
        case 0: KC_TRY(launch_emit<1>(ea, lst, cnt, st)); break;
        case 1: KC_TRY(launch_emit<2>(ea, lst, cnt, st)); break;
        case 2: KC_TRY(launch_emit<4>(ea, lst, cnt, st)); break;
        case 3: KC_TRY(launch_emit<8>(ea, lst, cnt, st)); break;
        case 4: KC_TRY(launch_emit<12>(ea, lst, cnt, st)); break;
        case 5: KC_TRY(launch_emit<16>(ea, lst, cnt, st)); break;
        case 6: KC_TRY(launch_emit<24>(ea, lst, cnt, st)); break;
        case 7: KC_TRY(launch_emit<32>(ea, lst, cnt, st)); break;
        case 8: KC_TRY((launch_emit<48, true>(ea, lst, cnt, st))); break;
        case 9: KC_TRY((launch_emit<64, true>(ea, lst, cnt, st))); break;
      }
    }
    return KC_OK;
  }
  if (c.root_features) {
    k_scatter_features<<<(R * 4 + 255) / 256, 256, 0, st>>>(R, c.roots, feat, c.root_features);
    KC_HIP(hipGetLastError());
  }

  // ---- schedule
  KC_TRY(ev_sched.start(st));
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
  // Split thresholds are set per word class: each class is its own
  // persistent launch, so each has its own tail to keep short.
  int32_t* hist;
  KC_TRY(scr.get(&hist, KC_NCLASS * KC_LOGW_BINS));
  KC_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * KC_NCLASS * KC_LOGW_BINS, st));
  k_sched_logw<<<(R + 255) / 256, 256, 0, st>>>(R, c.k, c.roots, c.vk, ri.s, ri.cls, pred, logw, hist);
  KC_HIP(hipGetLastError());
  std::vector<int32_t> hh(KC_NCLASS * KC_LOGW_BINS);
  KC_HIP(hipMemcpyAsync(hh.data(), hist, sizeof(int32_t) * hh.size(), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  const int slots = kc_device_cus() * 4;
  // split policy: shares of the class's estimated work (2) or fixed counts (1)
  const int policy = opt && opt->split_policy > 0 ? opt->split_policy : (learned ? 2 : 1);
  if (policy > 2) return KC_EINVAL;
  ClassBins cb;
  for (int cl = 0; cl < KC_NCLASS; ++cl) {
    const int32_t* h = hh.data() + cl * KC_LOGW_BINS;
    int lo_bin = KC_LOGW_BINS, hi_bin = KC_LOGW_BINS;
    if (opt && opt->split_threshold > 0.f) {
      lo_bin = (int)(opt->split_threshold * KC_LOGW_SCALE);
      hi_bin = (int)((opt->split_threshold + 4.0f) * KC_LOGW_SCALE);
    } else if (policy == 2) {
      // the class's estimated work; a root heavier than 1/(8 slots) of it is
      // split once, one heavier than 64 such shares twice
      double tot = 0.0;
      for (int b = 0; b < KC_LOGW_BINS; ++b) tot += (double)h[b] * exp((b + 0.5) / KC_LOGW_SCALE);
      double target = tot / (8.0 * slots);
      if (target > 1.0) {
        lo_bin = (int)(log(target) * KC_LOGW_SCALE) + 1;
        hi_bin = (int)(log(target * 64.0) * KC_LOGW_SCALE) + 1;
      }
    } else {
      // fixed counts: in each class the slots/4 roots of highest key are
      // split twice and the next 4 x slots once
      const int64_t n2 = slots / 4, n1 = (int64_t)slots * 4;
      int64_t cum = 0;
      for (int b = KC_LOGW_BINS - 1; b >= 0; --b) {
        cum += h[b];
        if (hi_bin == KC_LOGW_BINS && cum >= n2) hi_bin = b + 1;
        if (cum >= n2 + n1) { lo_bin = b + 1; break; }
      }
      if (lo_bin > hi_bin) lo_bin = hi_bin;
    }
    cb.lo[cl] = lo_bin;
    cb.hi[cl] = hi_bin;
  }
  const int force = opt ? opt->split : 0;
  k_sched_depth<<<(R + 255) / 256, 256, 0, st>>>(R, c.k, c.roots, c.vk, ri.cls, logw, cb, force, depth);
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
  sp.vk = c.vk;
  sp.noprune = opt && (opt->disable & KC_NO_PRUNE) ? 1 : 0;
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
  KC_TRY(ev_sched.stop(st));

  // ---- listing: one persistent launch per bitmap class, heaviest first
  unsigned long long* heads;
  KC_TRY(scr.get(&heads, KC_NCLASS));
  unsigned long long* cls_ctr;
  KC_TRY(scr.get(&cls_ctr, KC_NCTR * KC_NCLASS));
  ListArgs las[KC_NCLASS];
  int nws[KC_NCLASS];
  for (int cl = 0; cl < KC_NCLASS; ++cl) {
    int32_t lo = boff[cl * 64], hi = boff[(cl + 1) * 64];
    ListArgs& la = las[cl];
    la.roots = c.roots;
    la.ri = ri;
    la.B = B;
    la.Bin = Bin;
    la.perm = perm;
    la.color = color;
    la.tasks = tasks_sorted + lo;
    la.ntasks = hi - lo;
    la.head = heads + cl;
    nws[cl] = opt && opt->waves_per_root > 0
                  ? opt->waves_per_root
                  : (kWClass[cl] >= 24 ? 16 : (kWClass[cl] >= 8 ? 8 : (kWClass[cl] >= 4 ? 4 : 1)));
    la.chunk = opt && opt->chunk > 0 ? opt->chunk : (kWClass[cl] >= 8 ? 1 : 8);
    la.k = c.k;
    la.vk = c.vk;
    la.root_count = c.root_count;
    {
      const int cap = pv ? 64 : 128;  // two-word re-encoding only when counting
      const int want = opt ? opt->compress : 0;  // 0 = auto: the cap; < 0 = off
      la.cmax = want == 0 ? cap : (want < 0 ? 0 : (want > cap ? cap : want));
    }
    la.clev = opt && opt->compress_level > 0 ? opt->compress_level : 4;
    la.noprune = opt && (opt->disable & KC_NO_PRUNE) ? 1 : 0;
    la.count = c.count;
    la.pv = c.pv;
    la.counters = cls_ctr + KC_NCTR * cl;
    la.root_work = c.root_work;
    la.root_isect = c.root_isect;
    la.flags = c.flags;
  }
  if (c.capture) {
    // a prepared call: hand the listing phase over to be captured and replayed
    BitcolReplay* rp = new BitcolReplay;
    rp->heads = heads;
    rp->cls_ctr = cls_ctr;
    rp->counters = c.counters;
    for (int cl = 0; cl < KC_NCLASS; ++cl) {
      rp->la[cl] = las[cl];
      rp->used[cl] = las[cl].ntasks > 0;
      if (rp->used[cl]) {
        const int st2 = resolve_list_class(las[cl], cl, nws[cl], pv, &rp->ll[cl]);
        if (st2 != KC_OK) {
          delete rp;
          return st2;
        }
      }
    }
    c.capture->state = rp;
    c.capture->launch = bitcol_replay_launch;
    c.capture->destroy = bitcol_replay_destroy;
    return KC_OK;
  }
  if (c.size_only) return KC_OK;  // every allocation of the call is made
  KC_HIP(hipMemsetAsync(heads, 0, sizeof(unsigned long long) * KC_NCLASS, st));
  KC_TRY(ev_list.start(st));
  int launches = 0;
  EventPair ev_cls[KC_NCLASS];
  KC_HIP(hipMemsetAsync(cls_ctr, 0, sizeof(unsigned long long) * KC_NCTR * KC_NCLASS, st));
  // One persistent kernel per word class, heaviest class first.  They either
  // follow each other on the call's stream, or run concurrently on streams of
  // their own (default priority) so that one class's tail overlaps the next
  // class's work.  Auto: the learned schedule splits every class's heavy
  // roots by its own predicted work and leaves no long tails, so its classes
  // run in sequence; the degree schedule's tails are overlapped.
  const int cmode = opt && opt->class_streams > 0 ? opt->class_streams : (learned ? 1 : 2);
  struct Streams {
    hipStream_t s[KC_NCLASS] = {};
    hipEvent_t done[KC_NCLASS] = {};
    ~Streams() {
      for (int i = 0; i < KC_NCLASS; ++i) {
        if (done[i]) (void)hipEventDestroy(done[i]);
        if (s[i]) (void)hipStreamDestroy(s[i]);
      }
    }
  } cs;
  struct EvGuard {
    hipEvent_t e = nullptr;
    ~EvGuard() {
      if (e) (void)hipEventDestroy(e);
    }
  } ready;
  if (cmode == 2) {
    KC_HIP(hipEventCreateWithFlags(&ready.e, hipEventDisableTiming));
    KC_HIP(hipEventRecord(ready.e, st));
  }
  for (int cl = KC_NCLASS - 1; cl >= 0; --cl) {
    if (las[cl].ntasks <= 0) continue;
    hipStream_t ls = st;
    if (cmode == 2) {
      KC_HIP(hipStreamCreateWithFlags(&cs.s[cl], hipStreamNonBlocking));
      KC_HIP(hipEventCreateWithFlags(&cs.done[cl], hipEventDisableTiming));
      KC_HIP(hipStreamWaitEvent(cs.s[cl], ready.e, 0));
      ls = cs.s[cl];
    }
    KC_TRY(ev_cls[cl].init(timed));
    KC_TRY(ev_cls[cl].start(ls));
    KC_TRY(launch_list_class(las[cl], cl, nws[cl], pv, ls));
    KC_TRY(ev_cls[cl].stop(ls));
    if (cmode == 2) {
      KC_HIP(hipEventRecord(cs.done[cl], ls));
      KC_HIP(hipStreamWaitEvent(st, cs.done[cl], 0));
    }
    launches++;
  }
  k_add_counters<<<1, 64, 0, st>>>(cls_ctr, KC_NCLASS, c.counters);
  KC_HIP(hipGetLastError());
  KC_TRY(ev_list.stop(st));
  if (c.stats) {
    c.stats->stage_ms += ev_stage.ms();
    c.stats->sched_ms += ev_sched.ms();
    c.stats->list_ms += ev_list.ms();
    c.stats->list_launches += launches;
    c.stats->n_tasks += NT;
    unsigned long long hc[KC_NCTR * KC_NCLASS];
    KC_HIP(hipMemcpyAsync(hc, cls_ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    for (int cl = 0; cl < KC_NCLASS; ++cl) {
      if (ev_cls[cl].a) c.stats->class_ms[cl] = ev_cls[cl].ms();
      c.stats->class_work[cl] = hc[KC_NCTR * cl + 2];
      c.stats->class_tasks[cl] = boff[(cl + 1) * 64] - boff[cl * 64];
    }
  }
  return KC_OK;
}
