// kc_sdegree.hip -- SDegree (Alg. 5, Sec. 6.2) on gfx950.
//
// Work items are roots u with d+_u >= k-1 (NodeParallel, Sec. 9) or, for the
// roots whose estimated work is heaviest, a root with its first candidate x
// fixed (the edge (u, x): EdgeParallel, Sec. 10), so that no single heavy root
// holds one wave for the whole run.  A persistent one-wave workgroup takes
// items from a queue.  The candidate set C of every recursion level is a
// sorted list of vertex ids held in LDS (or, for very large out-degrees, in a
// per-workgroup slice of device memory).  The merge join of Alg. 5 -- C' =
// N+(x) intersected with C -- is done with 64 lanes at a time: the lanes load
// 64 consecutive entries of the sorted list N+(x) (one coalesced load), each
// lane looks its entry up in C by binary search, and a ballot compacts the
// hits into the next level's list in order (mbcnt gives each hit its slot).
// The part of N+(x) below min(C) is skipped with one binary search and the
// scan stops past max(C), so a join touches only the range where matches can
// occur.  Pruning follows Alg. 5: x is skipped when d+_x <= l-2, and a child
// list is entered only when it holds more than l-2 members.  Work is logged
// as |C| + d+_x per join, the cost term of Lemma 2.
//
// When counting, a level-2 node's joins are flattened: every candidate x of
// the node finds the range of N+(x) inside [min C, max C] (two binary
// searches), the ranges are laid end to end, and each lane takes every 64th
// entry of the concatenation, looks it up in C and counts the hits.  All
// lanes stay busy whatever the lengths of the lists, and the loads of one
// pass are independent of each other.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "kc_internal.h"

#define SD_NCLASS 6
// out-lists of at most this many entries are read whole by a join instead of
// locating the range that can match by binary search
#define SD_WHOLE_LIST 64
static const int kSClass[SD_NCLASS] = {64, 256, 1024, 4096, 16384, 65536};

__device__ __forceinline__ int sd_class_of(int s) {
  if (s <= 64) return 0;
  if (s <= 256) return 1;
  if (s <= 1024) return 2;
  if (s <= 4096) return 3;
  if (s <= 16384) return 4;
  if (s <= 65536) return 5;
  return -1;
}

struct SdArgs {
  const int32_t* drp;
  const int32_t* dcol;
  const int32_t* roots;
  const uint64_t* tasks;  // schedule order: (root index << 32) | (position of the fixed first candidate + 1, or 0)
  int32_t ntasks;
  unsigned long long* head;
  int chunk;
  int k;                  // maximum k (memory layout)
  const int32_t* vk;      // per-vertex k (nullable)
  unsigned long long* root_count;
  int SMAX;
  uint32_t* gscratch;     // per-workgroup memory when the lists do not fit LDS
  size_t block_words;
  unsigned long long* count;
  unsigned long long* pv;
  unsigned long long* counters;
  uint64_t* root_work;
  uint64_t* root_isect;
  int* flags;
  kc_emit e;              // listing output (EMIT instances)
  int noprune;            // ablation: no d+ <= l-2 skip; a child with any member is entered
  uint16_t* pool;         // out-neighbour reduction: per-workgroup pool of reduced lists
  int64_t pool_cap;       // its entries per workgroup
};

// Memory of one workgroup (words): list[K][SMAX] | lidx[K][SMAX] (per-vertex)
// | cnt[SMAX] u64 (per-vertex) | cur[K] | size[K] | chosen[K] | tot[K] u64
static size_t sd_words(int k, int smax, bool pv) {
  size_t K = (size_t)k;
  return K * smax * (pv ? 2 : 1) + (pv ? 2 * (size_t)smax : 0) + 5 * K + 8;
}

__device__ __forceinline__ int sd_lower_bound(const int32_t* a, int lo, int hi, int32_t x) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Adds a launch's work totals (per lane) and clique count (lane 0) to the
// device counters, once per wave.
__device__ __forceinline__ void sd_flush_counters(const SdArgs& a, int lane, uint64_t nodes, uint64_t isect,
                                                  uint64_t work, uint64_t count, bool ovf) {
  const uint64_t wn = kc_wave_sum_u64(nodes), wi = kc_wave_sum_u64(isect), ww = kc_wave_sum_u64(work);
  if (lane == 0) {
    if (wn) atomicAdd(&a.counters[0], (unsigned long long)wn);
    if (wi) atomicAdd(&a.counters[1], (unsigned long long)wi);
    if (ww) atomicAdd(&a.counters[2], (unsigned long long)ww);
    kc_add_checked(a.count, count, a.flags);
    if (ovf) atomicOr(a.flags, KC_FLAG_OVERFLOW);
  }
}

// EMIT: write every clique found (the emit step of Alg. 5: R + {x, y} for
// each hit y of a join at l = 2), rows reserved per 64-entry chunk with one
// atomic; `chosen` then holds the vertex ids of R.
template <bool PV, bool EMIT>
__global__ __launch_bounds__(64) void k_sdegree_list(SdArgs a) {
  extern __shared__ uint32_t lds[];
  uint32_t* mem = a.gscratch ? a.gscratch + (size_t)blockIdx.x * a.block_words : lds;
  const int K = a.k;
  const int SM = a.SMAX;
  int32_t* list = (int32_t*)mem;
  int32_t* lidx = list + (size_t)K * SM;
  unsigned long long* cnt = (unsigned long long*)(lidx + (PV ? (size_t)K * SM : 0));
  int32_t* cur = (int32_t*)(cnt + (PV ? SM : 0));
  int32_t* size = cur + K;
  int32_t* chosen = size + K;
  unsigned long long* tot = (unsigned long long*)(((uintptr_t)(chosen + K) + 7) & ~(uintptr_t)7);
  const int lane = threadIdx.x;
  __shared__ int32_t sh_task[2];
  __shared__ int32_t fl_lo[64], fl_off[65];  // flattened level-2 joins: range starts and offsets

  uint64_t my_nodes = 0, my_isect = 0, my_work = 0;  // per lane, this task
  // the launch's totals (per lane; the count on lane 0), added to the device
  // counters once at the end rather than per task
  uint64_t run_nodes = 0, run_isect = 0, run_work = 0, run_count = 0;
  bool run_ovf = false;
  for (;;) {
    if (lane == 0) {
      unsigned long long t = atomicAdd(a.head, (unsigned long long)a.chunk);
      sh_task[0] = (int32_t)(t < (unsigned long long)a.ntasks ? t : a.ntasks);
      long long e = (long long)t + a.chunk;
      sh_task[1] = (int32_t)(e < a.ntasks ? e : a.ntasks);
    }
    __syncthreads();
    const int32_t t_lo = sh_task[0], t_hi = sh_task[1];
    __syncthreads();
    if (t_lo >= t_hi) break;
    for (int32_t ti = t_lo; ti < t_hi; ++ti) {
      const uint64_t task = a.tasks[ti];
      const int32_t r = (int32_t)(task >> 32);
      const int32_t xp1 = (int32_t)(uint32_t)task;  // 0: the whole root
      const int32_t u = a.roots[r];
      const int32_t b0 = a.drp[u];
      const int32_t s0 = a.drp[u + 1] - b0;
      const int kt = kc_vk(a.vk, u, a.k);
      for (int i = lane; i < s0; i += 64) {
        list[i] = a.dcol[b0 + i];
        if (PV) {
          lidx[i] = i;
          cnt[i] = 0;
        }
      }
      // level 0 walks candidates [cur, end0): all of N+(u), or only the
      // fixed one (the root's own call is then counted by the split pass)
      const int end0 = xp1 ? xp1 : s0;
      if (lane == 0) {
        cur[0] = xp1 ? xp1 - 1 : 0;
        size[0] = s0;
        tot[0] = 0;
      }
      __syncthreads();
      my_nodes += (lane == 0 && !xp1);
      const int L0 = kt - 1;
      int d = 0;
      for (;;) {
        const int l = L0 - d;
        const int sz = size[d];
        const int c = cur[d];
        const int end = d == 0 ? end0 : sz;
        if (c >= end) {
          if (d == 0) break;
          unsigned long long T = tot[d];
          if (lane == 0) {
            tot[d - 1] += T;
            if (PV && T) atomicAdd(&cnt[chosen[d - 1]], T);
          }
          kc_wave_lds_sync();
          d--;
          continue;
        }
        int32_t* C = list + (size_t)d * SM;
        if (!PV && !EMIT && l == 2) {
          // A level-2 node, counted with flattened joins (same pruning,
          // joins and work as one join per candidate).
          const int32_t cmin = C[0], cmax = C[sz - 1];
          uint32_t hits = 0;
          for (int b = c; b < end; b += 64) {
            const int idx = b + lane;
            int lo = 0, len = 0;
            if (idx < end) {
              const int32_t x = C[idx];
              const int32_t xb = a.drp[x], xe = a.drp[x + 1];
              const int dx = xe - xb;
              if (dx > 0 || a.noprune) {
                my_isect++;
                my_work += (uint64_t)sz + (uint64_t)dx;
                // a short list is taken whole (its entries outside
                // [min C, max C] find no match): one load instead of two
                // chains of dependent loads
                int l0 = xb, l1 = xe;
                if (dx > SD_WHOLE_LIST) {
                  int h0 = xe;
                  while (l0 < h0) {
                    const int mid = (l0 + h0) >> 1;
                    if (a.dcol[mid] < cmin) l0 = mid + 1; else h0 = mid;
                  }
                  l1 = l0;
                  int h1 = xe;
                  while (l1 < h1) {
                    const int mid = (l1 + h1) >> 1;
                    if (a.dcol[mid] <= cmax) l1 = mid + 1; else h1 = mid;
                  }
                }
                lo = l0;
                len = l1 - l0;
              }
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
              const int y = __shfl_up(incl, o, 64);
              if (lane >= o) incl += y;
            }
            const int total_len = __shfl(incl, 63, 64);
            fl_lo[lane] = lo;
            fl_off[lane] = incl - len;
            if (lane == 63) fl_off[64] = incl;
            kc_wave_lds_sync();
            for (int t0 = 0; t0 < total_len; t0 += 128) {
              // two entries per lane per pass, both loads issued first
              const int ta = t0 + lane, tb = t0 + 64 + lane;
              int32_t ya = 0x7fffffff, yb = 0x7fffffff;
              if (ta < total_len) {
                int p0 = 0, p1 = 65;
                while (p0 < p1) {
                  const int mid = (p0 + p1) >> 1;
                  if (fl_off[mid] <= ta) p0 = mid + 1; else p1 = mid;
                }
                ya = a.dcol[fl_lo[p0 - 1] + (ta - fl_off[p0 - 1])];
              }
              if (tb < total_len) {
                int p0 = 0, p1 = 65;
                while (p0 < p1) {
                  const int mid = (p0 + p1) >> 1;
                  if (fl_off[mid] <= tb) p0 = mid + 1; else p1 = mid;
                }
                yb = a.dcol[fl_lo[p0 - 1] + (tb - fl_off[p0 - 1])];
              }
              if (ta < total_len) {
                const int q = sd_lower_bound(C, 0, sz, ya);
                hits += (q < sz && C[q] == ya);
              }
              if (tb < total_len) {
                const int q = sd_lower_bound(C, 0, sz, yb);
                hits += (q < sz && C[q] == yb);
              }
            }
            kc_wave_lds_sync();  // the ranges are rewritten by the next batch
          }
          const uint64_t T2 = kc_wave_sum_u64(hits);
          if (lane == 0) {
            tot[d] += (unsigned long long)T2;
            cur[d] = end;
          }
          kc_wave_lds_sync();
          continue;
        }
        const int32_t x = C[c];
        const int xi = PV ? lidx[(size_t)d * SM + c] : 0;
        if (lane == 0) cur[d] = c + 1;
        kc_wave_lds_sync();
        const int32_t xb = a.drp[x], xe = a.drp[x + 1];
        const int dx = xe - xb;
        if (dx <= l - 2 && !a.noprune) continue;
        my_isect += (lane == 0);
        my_work += lane == 0 ? (uint64_t)sz + (uint64_t)dx : 0u;
        // merge join N+(x) with C
        const int32_t cmin = C[0], cmax = C[sz - 1];
        // first entry of N+(x) that can match (a short list is read whole)
        int start = xb;
        if (dx > SD_WHOLE_LIST) {
          int lo = xb, hi = xe;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (a.dcol[mid] < cmin) lo = mid + 1; else hi = mid;
          }
          start = lo;
        }
        int32_t* Cn = list + (size_t)(d + 1) * SM;
        int32_t* Ln = lidx + (size_t)(d + 1) * SM;
        int m = 0;
        int lo_pos = 0;
        for (int i0 = start; i0 < xe; i0 += 64) {
          const int i = i0 + lane;
          const int32_t y = i < xe ? a.dcol[i] : 0x7fffffff;
          const int32_t yfirst = __shfl(y, 0, 64);
          if (yfirst > cmax) break;
          int p = -1;
          if (y <= cmax) {
            int q = sd_lower_bound(C, lo_pos, sz, y);
            if (q < sz && C[q] == y) p = q;
          }
          const bool hit = p >= 0;
          const uint64_t mk = kc_ballot(hit);
          if (l == 2) {
            if (PV && hit) atomicAdd(&cnt[lidx[(size_t)d * SM + p]], 1ull);
            if (EMIT && mk) {
              unsigned long long base = 0;
              if (lane == 0) base = atomicAdd(a.e.pos, (unsigned long long)__popcll(mk));
              base = (unsigned long long)__shfl((long long)base, 0, 64);
              const unsigned long long row = base + (unsigned long long)kc_mbcnt(mk);
              if (hit && row < (unsigned long long)a.e.cap) {
                int32_t* o = a.e.out + (int64_t)row * a.k;
                o[0] = u;
                for (int q = 0; q < d; ++q) o[1 + q] = chosen[q];
                o[1 + d] = x;
                o[2 + d] = y;
              }
            }
          } else if (hit) {
            const int o = m + kc_mbcnt(mk);
            Cn[o] = y;
            if (PV) Ln[o] = lidx[(size_t)d * SM + p];
          }
          m += __popcll(mk);
          // entries of the next chunk are larger than every entry here
          const int32_t ylast = __shfl(y, 63, 64);
          if (ylast > cmax) break;
          lo_pos = sd_lower_bound(C, lo_pos, sz, ylast);
        }
        if (l == 2) {
          if (lane == 0) {
            tot[d] += (unsigned long long)m;
            if (PV && m) atomicAdd(&cnt[xi], (unsigned long long)m);
          }
          kc_wave_lds_sync();
        } else if (a.noprune ? m > 0 : m > l - 2) {
          if (lane == 0) {
            chosen[d] = EMIT ? x : xi;
            size[d + 1] = m;
            cur[d + 1] = 0;
            tot[d + 1] = 0;
          }
          kc_wave_lds_sync();
          d++;
          my_nodes += (lane == 0);
        }
      }
      __syncthreads();
      const unsigned long long T = tot[0];
      if (lane == 0 && T) {
        run_ovf |= run_count + T < run_count;
        run_count += T;
        if (a.root_count) kc_add_checked(&a.root_count[u], T, a.flags);
        if (PV) kc_add_checked(&a.pv[u], T, a.flags);
      }
      if (PV)
        for (int i = lane; i < s0; i += 64) {
          unsigned long long cc = cnt[i];
          if (cc) kc_add_checked(&a.pv[a.dcol[b0 + i]], cc, a.flags);
        }
      run_nodes += my_nodes;
      run_isect += my_isect;
      run_work += my_work;
      if (a.root_isect || a.root_work) {
        const uint64_t wi = kc_wave_sum_u64(my_isect), ww = kc_wave_sum_u64(my_work);
        if (lane == 0) {
          if (a.root_isect && wi) atomicAdd((unsigned long long*)&a.root_isect[u], (unsigned long long)wi);
          if (a.root_work && ww) atomicAdd((unsigned long long*)&a.root_work[u], (unsigned long long)ww);
        }
      }
      my_nodes = my_isect = my_work = 0;
      __syncthreads();
    }
  }
  sd_flush_counters(a, lane, run_nodes, run_isect, run_work, run_count, run_ovf);
}


// ---- SDegree with the out-neighbour reduction (Sec. 7.2) ----------------
// The recursion of a work item runs on the DAG G_u induced by N+(u): vertex i
// of G_u is position i of N+(u) (ascending ids, in LDS) and its out-list is
// L_i = {j : N+(u)[j] in N+(x_i)}, stored as 16-bit positions in a
// per-workgroup pool in device memory.  A whole-root item stages every L_i;
// an edge item (u, x) stages L_x and the lists of its members (every deeper
// candidate set lies inside L_x).  Staging is flattened over 64 candidates as
// the level-2 joins are: each candidate's range of N+(x_i) inside
// [min N+(u), max N+(u)] is found, the ranges are laid end to end, each lane
// takes one entry and finds it in N+(u) by binary search, and the hits are
// compacted in entry order, so each list's members stay together.
// The candidate sets of the recursion are position lists, each with a bitmap
// (LDS); a join of L_x with C is one bitmap test per entry of L_x.  The sets
// are kept in the order their members are found (neither the counts nor the
// logged work depend on it).  Pruning and work follow Alg. 5 on G_u: x is
// skipped when |L_x| <= l-2 and a join costs |C| + |L_x| (Lemma 2 on G_u).

// LDS of a reduced-SDegree workgroup (32-bit words): ids[SM] | lst[SM] |
// lln[SM] | clist[K][SM] u16 | bm[K][SM/32] | cur[K] | size[K] | chosen[K] |
// tot[K] u64 | cnt[SM] u64 (per-vertex output)
static size_t sdr_words(int k, int smax, bool pv) {
  const size_t K = (size_t)k, S = (size_t)smax;
  return 3 * S + K * S / 2 + K * (S / 32) + 5 * K + 8 + (pv ? 2 * S : 0);
}

// Stages the reduced lists of the candidates cand[0..nc) (positions of
// N+(u)) into the pool from `top`, and records where each one starts.
__device__ void sdr_stage(const SdArgs& a, const int32_t* ids, int s, const uint16_t* cand, int nc,
                          int32_t* lst, int32_t* lln, uint16_t* pool, int64_t& top, int lane, int32_t* fl_lo,
                          int32_t* fl_off, int32_t* fl_cnt) {
  const int32_t vmin = ids[0], vmax = ids[s - 1];
  for (int b = 0; b < nc; b += 64) {
    const int idx = b + lane;
    int lo = 0, len = 0, ci = -1;
    if (idx < nc) {
      ci = cand[idx];
      const int32_t x = ids[ci];
      const int32_t xb = a.drp[x], xe = a.drp[x + 1];
      int l0 = xb, l1 = xe;
      if (xe - xb > SD_WHOLE_LIST) {  // a short list is taken whole
        int h0 = xe;
        while (l0 < h0) {
          const int mid = (l0 + h0) >> 1;
          if (a.dcol[mid] < vmin) l0 = mid + 1; else h0 = mid;
        }
        l1 = l0;
        int h1 = xe;
        while (l1 < h1) {
          const int mid = (l1 + h1) >> 1;
          if (a.dcol[mid] <= vmax) l1 = mid + 1; else h1 = mid;
        }
      }
      lo = l0;
      len = l1 - l0;
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, 63, 64);
    fl_lo[lane] = lo;
    fl_off[lane] = incl - len;
    if (lane == 63) fl_off[64] = incl;
    fl_cnt[lane] = 0;
    kc_wave_lds_sync();
    int64_t base = top;
    for (int t0 = 0; t0 < total; t0 += 64) {
      const int t = t0 + lane;
      int q = -1, seg = 0;
      if (t < total) {
        int p0 = 0, p1 = 65;
        while (p0 < p1) {
          const int mid = (p0 + p1) >> 1;
          if (fl_off[mid] <= t) p0 = mid + 1; else p1 = mid;
        }
        seg = p0 - 1;
        const int32_t y = a.dcol[fl_lo[seg] + (t - fl_off[seg])];
        const int r = sd_lower_bound(ids, 0, s, y);
        if (r < s && ids[r] == y) q = r;
      }
      const bool hit = q >= 0;
      const uint64_t mk = kc_ballot(hit);
      if (hit) {
        const int64_t o = base + kc_mbcnt(mk);
        if (o < a.pool_cap) pool[o] = (uint16_t)q;  // the bound holds for a simple graph
        atomicAdd(&fl_cnt[seg], 1);
      }
      base += __popcll(mk);
    }
    kc_wave_lds_sync();
    const int cnt = fl_cnt[lane];
    int inc2 = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc2, o, 64);
      if (lane >= o) inc2 += y;
    }
    if (idx < nc) {
      lst[ci] = (int32_t)(top + inc2 - cnt);
      lln[ci] = cnt;
    }
    top = base;
    kc_wave_lds_sync();
  }
}

__device__ __forceinline__ bool sdr_bit(const uint32_t* bm, int e) { return (bm[e >> 5] >> (e & 31)) & 1u; }

// PV: per-vertex participation (each hit credits its own vertex and its
// candidate, subtree totals flow to the vertices chosen above, as in
// k_sdegree_list); EMIT: every clique written as k vertex ids.
template <bool PV, bool EMIT>
__global__ __launch_bounds__(64) void k_sdegree_reduced(SdArgs a) {
  extern __shared__ uint32_t lds[];
  const int K = a.k;
  const int SM = a.SMAX;
  const int SMW = SM >> 5;
  int32_t* ids = (int32_t*)lds;
  int32_t* lst = ids + SM;
  int32_t* lln = lst + SM;
  uint16_t* clist = (uint16_t*)(lln + SM);
  uint32_t* bm = (uint32_t*)(clist + (size_t)K * SM);
  int32_t* cur = (int32_t*)(bm + (size_t)K * SMW);
  int32_t* size = cur + K;
  int32_t* chosen = size + K;  // positions of the vertices chosen above the current level
  unsigned long long* tot = (unsigned long long*)(((uintptr_t)(chosen + K) + 7) & ~(uintptr_t)7);
  unsigned long long* cnt = tot + K;
  uint16_t* pool = a.pool + (size_t)blockIdx.x * (size_t)a.pool_cap;
  const int lane = threadIdx.x;
  __shared__ int32_t sh_task[2];
  __shared__ int32_t fl_lo[64], fl_off[65], fl_cnt[64];

  uint64_t my_nodes = 0, my_isect = 0, my_work = 0;
  uint64_t run_nodes = 0, run_isect = 0, run_work = 0, run_count = 0;  // the launch's totals
  bool run_ovf = false;
  for (;;) {
    if (lane == 0) {
      unsigned long long t = atomicAdd(a.head, (unsigned long long)a.chunk);
      sh_task[0] = (int32_t)(t < (unsigned long long)a.ntasks ? t : a.ntasks);
      long long e = (long long)t + a.chunk;
      sh_task[1] = (int32_t)(e < a.ntasks ? e : a.ntasks);
    }
    __syncthreads();
    const int32_t t_lo = sh_task[0], t_hi = sh_task[1];
    __syncthreads();
    if (t_lo >= t_hi) break;
    for (int32_t ti = t_lo; ti < t_hi; ++ti) {
      const uint64_t task = a.tasks[ti];
      const int32_t r = (int32_t)(task >> 32);
      const int32_t xp1 = (int32_t)(uint32_t)task;  // 0: the whole root
      const int32_t u = a.roots[r];
      const int32_t b0 = a.drp[u];
      const int32_t s0 = a.drp[u + 1] - b0;
      const int kt = kc_vk(a.vk, u, a.k);
      for (int i = lane; i < s0; i += 64) {
        ids[i] = a.dcol[b0 + i];
        lst[i] = -1;
        lln[i] = 0;
        clist[i] = (uint16_t)i;  // level 0: every position
        if (PV) cnt[i] = 0;
      }
      for (int w = lane; w < SMW; w += 64) {
        const int lo = w * 32;
        bm[w] = lo >= s0 ? 0u : (s0 - lo >= 32 ? ~0u : ((1u << (s0 - lo)) - 1u));
      }
      __syncthreads();
      // the lists this item can join
      int64_t top = 0;
      if (xp1) {
        const uint16_t x0 = (uint16_t)(xp1 - 1);
        clist[SM] = x0;  // a one-entry candidate list (level 1's list is rebuilt below)
        kc_wave_lds_sync();
        sdr_stage(a, ids, s0, clist + SM, 1, lst, lln, pool, top, lane, fl_lo, fl_off, fl_cnt);
        __syncthreads();
        const int n0 = top > a.pool_cap ? 0 : lln[x0];
        const uint16_t* l0 = pool + lst[x0];
        sdr_stage(a, ids, s0, l0, n0, lst, lln, pool, top, lane, fl_lo, fl_off, fl_cnt);
      } else {
        sdr_stage(a, ids, s0, clist, s0, lst, lln, pool, top, lane, fl_lo, fl_off, fl_cnt);
      }
      __syncthreads();
      if (top > a.pool_cap) {
        if (lane == 0) atomicOr(a.flags, KC_FLAG_TOOBIG);
        continue;
      }
      const int end0 = xp1 ? xp1 : s0;
      if (lane == 0) {
        cur[0] = xp1 ? xp1 - 1 : 0;
        size[0] = s0;
        tot[0] = 0;
      }
      __syncthreads();
      my_nodes += (lane == 0 && !xp1);
      const int L0 = kt - 1;
      int d = 0;
      for (;;) {
        const int l = L0 - d;
        const int sz = size[d];
        const int c = cur[d];
        const int end = d == 0 ? end0 : sz;
        if (c >= end) {
          if (d == 0) break;
          const unsigned long long T = tot[d];
          if (lane == 0) {
            tot[d - 1] += T;
            if (PV && T) atomicAdd(&cnt[chosen[d - 1]], T);
          }
          kc_wave_lds_sync();
          d--;
          continue;
        }
        const uint16_t* C = clist + (size_t)d * SM;
        const uint32_t* B = bm + (size_t)d * SMW;
        if (l == 2) {
          // a level-2 node: the entries of its candidates' lists laid end to
          // end, one bitmap test each
          uint32_t hits = 0;
          for (int b = c; b < end; b += 64) {
            const int idx = b + lane;
            int lo = 0, len = 0;
            if (idx < end) {
              const int x = C[idx];
              const int nx = lln[x];
              if (nx > 0 || a.noprune) {
                my_isect++;
                my_work += (uint64_t)sz + (uint64_t)nx;
                lo = lst[x];
                len = nx;
              }
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
              const int y = __shfl_up(incl, o, 64);
              if (lane >= o) incl += y;
            }
            const int total_len = __shfl(incl, 63, 64);
            fl_lo[lane] = lo;
            fl_off[lane] = incl - len;
            if (lane == 63) fl_off[64] = incl;
            kc_wave_lds_sync();
            for (int t0 = 0; t0 < total_len; t0 += 64) {
              const int t = t0 + lane;
              bool hit = false;
              int e = 0, seg = 0;
              if (t < total_len) {
                int p0 = 0, p1 = 65;
                while (p0 < p1) {
                  const int mid = (p0 + p1) >> 1;
                  if (fl_off[mid] <= t) p0 = mid + 1; else p1 = mid;
                }
                seg = p0 - 1;
                e = pool[fl_lo[seg] + (t - fl_off[seg])];
                hit = sdr_bit(B, e);
              }
              hits += hit ? 1u : 0u;
              if (PV && hit) {
                atomicAdd(&cnt[e], 1ull);
                atomicAdd(&cnt[C[b + seg]], 1ull);
              }
              if (EMIT) {
                const uint64_t mk = kc_ballot(hit);
                if (mk) {
                  unsigned long long base = 0;
                  if (lane == 0) base = atomicAdd(a.e.pos, (unsigned long long)__popcll(mk));
                  base = (unsigned long long)__shfl((long long)base, 0, 64);
                  const unsigned long long row = base + (unsigned long long)kc_mbcnt(mk);
                  if (hit && row < (unsigned long long)a.e.cap) {
                    int32_t* o = a.e.out + (int64_t)row * a.k;
                    o[0] = u;
                    for (int q = 0; q < d; ++q) o[1 + q] = ids[chosen[q]];
                    o[1 + d] = ids[C[b + seg]];
                    o[2 + d] = ids[e];
                  }
                }
              }
            }
            kc_wave_lds_sync();
          }
          const uint64_t T2 = kc_wave_sum_u64(hits);
          if (lane == 0) {
            tot[d] += (unsigned long long)T2;
            cur[d] = end;
          }
          kc_wave_lds_sync();
          continue;
        }
        const int x = C[c];
        if (lane == 0) cur[d] = c + 1;
        kc_wave_lds_sync();
        const int nx = lln[x];
        if (nx <= l - 2 && !a.noprune) continue;
        my_isect += (lane == 0);
        my_work += lane == 0 ? (uint64_t)sz + (uint64_t)nx : 0u;
        // C' = L_x with C: bitmap tests, hits compacted into level d+1
        uint16_t* Cn = clist + (size_t)(d + 1) * SM;
        uint32_t* Bn = bm + (size_t)(d + 1) * SMW;
        for (int w = lane; w < SMW; w += 64) Bn[w] = 0u;
        kc_wave_lds_sync();
        const uint16_t* Lx = pool + lst[x];
        int m = 0;
        for (int i0 = 0; i0 < nx; i0 += 64) {
          const int i = i0 + lane;
          const int e = i < nx ? (int)Lx[i] : 0;
          const bool hit = i < nx && sdr_bit(B, e);
          const uint64_t mk = kc_ballot(hit);
          if (hit) {
            Cn[m + kc_mbcnt(mk)] = (uint16_t)e;
            atomicOr(&Bn[e >> 5], 1u << (e & 31));
          }
          m += __popcll(mk);
        }
        kc_wave_lds_sync();
        if (a.noprune ? m > 0 : m > l - 2) {
          if (lane == 0) {
            chosen[d] = x;
            size[d + 1] = m;
            cur[d + 1] = 0;
            tot[d + 1] = 0;
          }
          kc_wave_lds_sync();
          d++;
          my_nodes += (lane == 0);
        }
      }
      __syncthreads();
      const unsigned long long T = tot[0];
      if (lane == 0 && T) {
        run_ovf |= run_count + T < run_count;
        run_count += T;
        if (a.root_count) kc_add_checked(&a.root_count[u], T, a.flags);
        if (PV) kc_add_checked(&a.pv[u], T, a.flags);
      }
      if (PV)
        for (int i = lane; i < s0; i += 64) {
          const unsigned long long cc = cnt[i];
          if (cc) kc_add_checked(&a.pv[ids[i]], cc, a.flags);
        }
      run_nodes += my_nodes;
      run_isect += my_isect;
      run_work += my_work;
      if (a.root_isect || a.root_work) {
        const uint64_t wi = kc_wave_sum_u64(my_isect), ww = kc_wave_sum_u64(my_work);
        if (lane == 0) {
          if (a.root_isect && wi) atomicAdd((unsigned long long*)&a.root_isect[u], (unsigned long long)wi);
          if (a.root_work && ww) atomicAdd((unsigned long long*)&a.root_work[u], (unsigned long long)ww);
        }
      }
      my_nodes = my_isect = my_work = 0;
      __syncthreads();
    }
  }
  sd_flush_counters(a, lane, run_nodes, run_isect, run_work, run_count, run_ovf);
}

#define SD_LOGW_BINS 512
#define SD_LOGW_SCALE 8.0f

__device__ __forceinline__ float sd_log_binom(float n, float k) {
  if (k > n) return -1.0f;
  return lgammaf(n + 1.0f) - lgammaf(k + 1.0f) - lgammaf(n - k + 1.0f);
}

// Per root: candidate-list class and the degree schedule's work estimate
// log C(d+, k-1) (a histogram per class sets the split threshold).
__global__ void k_sd_est(int32_t R, const int32_t* __restrict__ roots, const int32_t* __restrict__ drp, int k0,
                         const int32_t* vk, int32_t* cls, float* logw, int32_t* hist, int32_t* cls_max, int* flags) {
  int32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  int32_t u = roots[r];
  const int k = kc_vk(vk, u, k0);
  int s = drp[u + 1] - drp[u];
  int c = sd_class_of(s);
  if (c < 0) {
    atomicOr(flags, KC_FLAG_TOOBIG);
    c = 0;
  }
  float lw = sd_log_binom((float)s, (float)(k - 1));
  if (!(lw > -1e30f)) lw = 0.f;
  cls[r] = c;
  logw[r] = lw;
  int b = (int)(lw * SD_LOGW_SCALE);
  b = b < 0 ? 0 : (b >= SD_LOGW_BINS ? SD_LOGW_BINS - 1 : b);
  atomicAdd(&hist[c * SD_LOGW_BINS + b], 1);
  atomicMax(&cls_max[c], s);
}

struct SdSplit {
  int thr[SD_NCLASS];  // split a root of this class when its estimate bin is >= thr
};

// Work items: a whole root, or, for a root to split, one item per candidate
// x of its top call that Alg. 5 does not skip (d+_x > k-3), in schedule
// order (heaviest first inside each class).  Mode 0 counts, mode 1 writes;
// the split roots' own calls are counted here.
__global__ void k_sd_tasks(int32_t R, const int32_t* __restrict__ roots, const int32_t* __restrict__ drp,
                           const int32_t* __restrict__ dcol, int k0, const int32_t* vk,
                           const int32_t* __restrict__ cls, const float* __restrict__ logw, SdSplit sp, int noprune,
                           int mode, unsigned long long* ntasks, uint64_t* tasks, int32_t* task_bin,
                           unsigned long long* counters) {
  const int lane = kc_lane();
  const int32_t wave = (int32_t)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / KC_WAVE);
  if (wave >= R) return;
  const int32_t r = wave;
  const int32_t u = roots[r];
  const int k = kc_vk(vk, u, k0);
  const int c = cls[r];
  const bool split = k >= 4 && (int)(logw[r] * SD_LOGW_SCALE) >= sp.thr[c];
  if (!split) {
    if (lane == 0) {
      unsigned long long o = atomicAdd(ntasks, 1ull);
      if (mode == 1) {
        tasks[o] = (uint64_t)(uint32_t)r << 32;
        task_bin[o] = c * 64 + 63 - kc_key_q(logw[r]);
      }
    }
    return;
  }
  const int32_t b0 = drp[u], s = drp[u + 1] - b0;
  for (int32_t i0 = 0; i0 < s; i0 += KC_WAVE) {
    const int32_t i = i0 + lane;
    int dx = 0;
    bool take = false;
    if (i < s) {
      const int32_t x = dcol[b0 + i];
      dx = drp[x + 1] - drp[x];
      take = noprune || dx > k - 3;
    }
    const uint64_t m = kc_ballot(take);
    unsigned long long base = 0;
    if (lane == 0 && m) base = atomicAdd(ntasks, (unsigned long long)__popcll(m));
    base = (unsigned long long)__shfl((long long)base, 0, 64);
    if (mode == 1 && take) {
      const unsigned long long o = base + (unsigned long long)kc_mbcnt(m);
      tasks[o] = ((uint64_t)(uint32_t)r << 32) | (uint64_t)(uint32_t)(i + 1);
      task_bin[o] = c * 64 + 63 - kc_key_q(sd_log_binom((float)(dx < s ? dx : s), (float)(k - 2)));
    }
  }
  if (mode == 1 && lane == 0) atomicAdd(&counters[0], 1ull);  // the root's own call
}

__global__ void k_sd_gather(const uint64_t* __restrict__ in, const int32_t* __restrict__ order, int32_t n,
                            uint64_t* out) {
  int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[order[i]];
}

__global__ void k_sd_add_counters(const unsigned long long* __restrict__ per_class, int ncls,
                                  unsigned long long* total) {
  int i = threadIdx.x;
  if (i < 3) {
    unsigned long long t = 0;
    for (int c = 0; c < ncls; ++c) t += per_class[3 * c + i];
    total[i] += t;
  }
}

int kc_list_sdegree(kc_list_ctx& c, kc_scratch& scr, hipStream_t st) {
  const int32_t R = c.nroots;
  if (R == 0) return KC_OK;
  const bool pv = c.pv != nullptr;
  const kc_options* opt = c.opt;
  int32_t *cls, *hist;
  float* logw;
  KC_TRY(scr.get(&cls, R));
  KC_TRY(scr.get(&logw, R));
  // per class: the estimate histogram, then the class's largest out-degree
  KC_TRY(scr.get(&hist, SD_NCLASS * SD_LOGW_BINS + SD_NCLASS));
  KC_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * (SD_NCLASS * SD_LOGW_BINS + SD_NCLASS), st));
  k_sd_est<<<(R + 255) / 256, 256, 0, st>>>(R, c.roots, c.drp, c.k, c.vk, cls, logw, hist,
                                            hist + SD_NCLASS * SD_LOGW_BINS, c.flags);
  KC_HIP(hipGetLastError());
  std::vector<int32_t> hh(SD_NCLASS * SD_LOGW_BINS + SD_NCLASS);
  int hflags = 0;
  KC_HIP(hipMemcpyAsync(hh.data(), hist, sizeof(int32_t) * hh.size(), hipMemcpyDeviceToHost, st));
  KC_HIP(hipMemcpyAsync(&hflags, c.flags, sizeof(int), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  if (hflags & KC_FLAG_TOOBIG) return KC_EUNSUPPORTED;
  // Which roots are split into one item per top-level candidate: per class,
  // those whose estimate exceeds 1/(8 slots) of the class's estimated total
  // (shares, the default), the slots/4 + 4 slots heaviest (fixed counts), or
  // those above an explicit threshold; never with split = -1.
  const int slots = kc_device_cus() * 4;
  const int policy = opt && opt->split_policy > 0 ? opt->split_policy : 2;
  if (policy > 2) return KC_EINVAL;
  SdSplit sp;
  for (int cl = 0; cl < SD_NCLASS; ++cl) {
    const int32_t* h = hh.data() + cl * SD_LOGW_BINS;
    int thr = SD_LOGW_BINS;
    if (opt && opt->split < 0) {
      thr = SD_LOGW_BINS + 1;
    } else if (opt && opt->split_threshold > 0.f) {
      thr = (int)(opt->split_threshold * SD_LOGW_SCALE);
    } else if (policy == 2) {
      double tot = 0.0;
      for (int b = 0; b < SD_LOGW_BINS; ++b) tot += (double)h[b] * exp((b + 0.5) / SD_LOGW_SCALE);
      const double target = tot / (8.0 * slots);
      if (target > 1.0) thr = (int)(log(target) * SD_LOGW_SCALE) + 1;
    } else {
      const int64_t want = (int64_t)slots / 4 + (int64_t)slots * 4;
      int64_t cum = 0;
      for (int b = SD_LOGW_BINS - 1; b >= 0; --b) {
        cum += h[b];
        if (cum >= want) { thr = b + 1; break; }
      }
    }
    sp.thr[cl] = thr;
  }
  const int noprune = opt && (opt->disable & KC_NO_PRUNE) ? 1 : 0;
  unsigned long long* ntask_dev;
  KC_TRY(scr.get(&ntask_dev, 2));
  KC_HIP(hipMemsetAsync(ntask_dev, 0, sizeof(unsigned long long), st));
  const unsigned tgrid = (unsigned)(((int64_t)R * KC_WAVE + 255) / 256);
  k_sd_tasks<<<tgrid, 256, 0, st>>>(R, c.roots, c.drp, c.dcol, c.k, c.vk, cls, logw, sp, noprune, 0, ntask_dev,
                                    nullptr, nullptr, c.counters);
  KC_HIP(hipGetLastError());
  unsigned long long nt_h = 0;
  KC_HIP(hipMemcpyAsync(&nt_h, ntask_dev, sizeof(nt_h), hipMemcpyDeviceToHost, st));
  KC_HIP(hipStreamSynchronize(st));
  if (nt_h >= (unsigned long long)INT32_MAX) return KC_EUNSUPPORTED;
  const int32_t NT = (int32_t)nt_h;
  uint64_t *tasks, *tasks_sorted;
  int32_t *task_bin, *order;
  KC_TRY(scr.get(&tasks, (size_t)NT + 1));
  KC_TRY(scr.get(&tasks_sorted, (size_t)NT + 1));
  KC_TRY(scr.get(&task_bin, (size_t)NT + 1));
  KC_TRY(scr.get(&order, (size_t)NT + 1));
  KC_HIP(hipMemsetAsync(ntask_dev, 0, sizeof(unsigned long long), st));
  k_sd_tasks<<<tgrid, 256, 0, st>>>(R, c.roots, c.drp, c.dcol, c.k, c.vk, cls, logw, sp, noprune, 1, ntask_dev,
                                    tasks, task_bin, c.counters);
  KC_HIP(hipGetLastError());
  const int NB = SD_NCLASS * 64;
  std::vector<int32_t> boff(NB + 1);
  KC_TRY(kc_bin_sort(task_bin, NT, NB, order, boff.data(), scr, st));
  if (NT > 0) {
    k_sd_gather<<<(NT + 255) / 256, 256, 0, st>>>(tasks, order, NT, tasks_sorted);
    KC_HIP(hipGetLastError());
  }
  unsigned long long* heads;
  KC_TRY(scr.get(&heads, SD_NCLASS));
  KC_HIP(hipMemsetAsync(heads, 0, sizeof(unsigned long long) * SD_NCLASS, st));
  // timing events only when statistics are asked for
  struct Events {
    hipEvent_t e0 = nullptr, e1 = nullptr, ce[SD_NCLASS][2] = {};
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      for (auto& p : ce)
        for (auto& e : p)
          if (e) (void)hipEventDestroy(e);
    }
  } ev;
  const bool timed = c.stats != nullptr && !c.size_only;
  unsigned long long* cls_ctr;
  KC_TRY(scr.get(&cls_ctr, 3 * SD_NCLASS));
  KC_HIP(hipMemsetAsync(cls_ctr, 0, sizeof(unsigned long long) * 3 * SD_NCLASS, st));
  if (timed) {
    KC_HIP(hipEventCreate(&ev.e0));
    KC_HIP(hipEventCreate(&ev.e1));
    KC_HIP(hipEventRecord(ev.e0, st));
  }
  int launches = 0;
  for (int cl = SD_NCLASS - 1; cl >= 0; --cl) {
    int32_t lo = boff[cl * 64], hi = boff[(cl + 1) * 64];
    if (hi <= lo) continue;
    if (timed) {
      KC_HIP(hipEventCreate(&ev.ce[cl][0]));
      KC_HIP(hipEventCreate(&ev.ce[cl][1]));
      KC_HIP(hipEventRecord(ev.ce[cl][0], st));
    }
    SdArgs a;
    a.drp = c.drp;
    a.dcol = c.dcol;
    a.roots = c.roots;
    a.tasks = tasks_sorted + lo;
    a.ntasks = hi - lo;
    a.head = heads + cl;
    a.chunk = c.opt && c.opt->chunk > 0 ? c.opt->chunk : (cl <= 1 ? 8 : 1);
    a.k = c.k;
    a.vk = c.vk;
    a.root_count = c.root_count;
    // lists sized for the class's largest out-degree (rounded up to 64), not
    // the class bound: the LDS per wave sets how many waves share a CU
    {
      const int cm = hh[SD_NCLASS * SD_LOGW_BINS + cl];
      const int fit = (cm + 63) & ~63;
      a.SMAX = fit > 0 && fit < kSClass[cl] ? fit : kSClass[cl];
    }
    a.count = c.count;
    a.pv = c.pv;
    a.counters = cls_ctr + 3 * cl;
    a.root_work = c.root_work;
    a.root_isect = c.root_isect;
    a.flags = c.flags;
    size_t words = sd_words(c.k, a.SMAX, pv);
    size_t bytes = 4 * words;
    a.e = c.emit ? *c.emit : kc_emit();
    a.noprune = c.opt && (c.opt->disable & KC_NO_PRUNE) ? 1 : 0;
    a.pool = nullptr;
    a.pool_cap = 0;
    if (c.reduce) {
      // G_u of up to 4096 vertices (the 4096-entry class; positions are
      // 16-bit): the reduced lists, at most SM (SM - 1) / 2 entries, in a
      // per-workgroup pool (16 MiB per workgroup at 4096)
      if (cl >= 4) return KC_EUNSUPPORTED;
      const size_t rbytes = 4 * sdr_words(c.k, a.SMAX, pv);
      int dev = 0, maxlds = 65536;
      KC_HIP(hipGetDevice(&dev));
      KC_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
      if (rbytes > (size_t)maxlds) return KC_EUNSUPPORTED;
      auto rfn = pv ? k_sdegree_reduced<true, false>
                    : (c.emit ? k_sdegree_reduced<false, true> : k_sdegree_reduced<false, false>);
      KC_HIP(hipFuncSetAttribute((const void*)rfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rbytes));
      int per_cu = 0;
      KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, rfn, 64, rbytes));
      int64_t rgrid = (int64_t)(per_cu < 1 ? 1 : per_cu) * kc_device_cus();
      if (rgrid > a.ntasks) rgrid = a.ntasks;
      if (rgrid < 1) rgrid = 1;
      a.gscratch = nullptr;
      a.block_words = 0;
      a.pool_cap = (int64_t)a.SMAX * (a.SMAX - 1) / 2 + 64;
      KC_TRY(scr.get(&a.pool, (size_t)a.pool_cap * (size_t)rgrid));
      if (c.size_only) continue;
      hipLaunchKernelGGL(rfn, dim3((unsigned)rgrid), dim3(64), rbytes, st, a);
      KC_HIP(hipGetLastError());
      if (timed) KC_HIP(hipEventRecord(ev.ce[cl][1], st));
      launches++;
      continue;
    }
    auto fn = pv ? k_sdegree_list<true, false> : (c.emit ? k_sdegree_list<false, true> : k_sdegree_list<false, false>);
    int64_t grid;
    size_t lds_bytes;
    if (bytes <= 64 * 1024) {
      a.gscratch = nullptr;
      a.block_words = 0;
      lds_bytes = bytes;
      KC_HIP(hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
      int per_cu = 0;
      KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64, lds_bytes));
      grid = (int64_t)(per_cu < 1 ? 1 : per_cu) * kc_device_cus();
    } else {
      // Lists in device memory are enabled for counting only: with per-vertex
      // or listing output they are refused until the cause of a GPU fault in
      // a run that exercised them is found.
      if (pv || c.emit) return KC_EUNSUPPORTED;
      grid = (int64_t)kc_device_cus() * 8;
      if (grid > a.ntasks) grid = a.ntasks;
      a.block_words = (words + 63) & ~(size_t)63;
      KC_TRY(scr.get(&a.gscratch, a.block_words * (size_t)grid));
      lds_bytes = 0;
    }
    if (grid > a.ntasks) grid = a.ntasks;
    if (grid < 1) grid = 1;
    if (c.size_only) continue;  // the scratch of every class is allocated above
    hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(64), lds_bytes, st, a);
    KC_HIP(hipGetLastError());
    if (timed) KC_HIP(hipEventRecord(ev.ce[cl][1], st));
    launches++;
  }
  if (c.size_only) return KC_OK;
  if (timed) KC_HIP(hipEventRecord(ev.e1, st));
  k_sd_add_counters<<<1, 64, 0, st>>>(cls_ctr, SD_NCLASS, c.counters);
  KC_HIP(hipGetLastError());
  if (c.stats) {
    float ms = 0.f;
    KC_HIP(hipEventSynchronize(ev.e1));
    KC_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    c.stats->list_ms += ms;
    c.stats->list_launches += launches;
    c.stats->n_tasks += NT;
    unsigned long long hc[3 * SD_NCLASS];
    KC_HIP(hipMemcpyAsync(hc, cls_ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
    KC_HIP(hipStreamSynchronize(st));
    for (int cl = 0; cl < SD_NCLASS; ++cl) {
      if (ev.ce[cl][0]) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev.ce[cl][0], ev.ce[cl][1]) == hipSuccess) c.stats->class_ms[cl] = t;
      }
      c.stats->class_work[cl] = hc[3 * cl + 2];
      c.stats->class_tasks[cl] = boff[(cl + 1) * 64] - boff[cl * 64];
    }
  }
  return KC_OK;
}
