// Sort path of the negative distance kernel (Sec. 3.2) and of the K2 part of
// the Laplacian (Sec. 3.3): for every slice,
//
//   t_m = -c' sum_n v_n |z_n - z_m|   over the union z = (y, x), v = (0, w),
//
// evaluated at the targets through the sorted order.  With A_<(m) and S_<(m)
// the sums of v and v z over the entries sorted before target m,
//
//   t_m = -c' [ z_m (2 A_< - A_tot) - (2 S_< - S_tot) ],
//
// which is Algorithm "fastsum_energy" regrouped (b_{m-1} and a_L (z_L - z_m)
// expanded into A and S); ties contribute 0 in either form.
//
// Implementation (per slice, all slices of a batch at once):
//   S1 hist     linear-in-value buckets over [c_min, c_max] (a monotone map, so
//               bucket order is value order); per bucket the count and the sums
//               of v and v (z - c_mid) as 64-bit fixed-point integers, so every
//               sum is exact and independent of the order of the atomics
//   S2 scan     bucket offsets and exclusive bucket prefixes of (A, S)
//   S3 scatter  (key, union index) pairs into their buckets
//   S4 groups   consecutive buckets holding about 2048..4096 entries are sorted
//               in LDS (stable LSD radix on 8-bit digits, wave ballots for the
//               in-wave ranks), ties ordered by union index, then a block scan
//               of the fixed-point (A, S) gives t at every target.  A group
//               larger than LDS is sorted by one workgroup streaming through
//               global memory with the same ranking.
// The order produced is the stable ascending order of the FP32 projections
// (ties by union index), i.e. the permutation sigma of Sec. 3.2.
//
// Derivative mode (gradients): the emitted value is d/dz_m of the sum,
// -c' (A_< - A_>) with strict inequalities (sign(0) = 0).  Targets have the lower
// union indices, so inside a run of equal keys they come before the sources:
// the exclusive prefix at a target is A_<, and A_> = A_tot - A_<= needs the sum
// A_= of the sources tied with it: D = -c' (2 A_< + A_= - A_tot).
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace ksum {

struct SortArgs {
  int32_t nsl, nb, G;
  int64_t L, M;
  const float *Z;
  const float *w;
  const SliceParams *params;
  const double *misc;
  uint32_t *hcnt;
  long long *hsum;
  long long *bpre;
  uint32_t *boff;
  long long *tot;
  unsigned long long *keys;
  unsigned long long *keys2;
  float *t;             // [nsl][M]
  int32_t *perm;        // [nsl][L] (already offset to the batch) or null
  double cneg;          // c' (c_d, or alpha c_d for the Laplacian)
  uint32_t *fail_count; // groups handed to the fallback kernel (zeroed by the scan kernel, or by the
                        // host-side launch when the buckets are reused)
  uint32_t *fail_list;  // [nsl * G] work items
  int4 *desc;           // [nsl][G] (first bucket, first entry, end entry, last bucket) of each group
  int32_t deriv;        // 0: t = the sums; 1: t = their derivatives at the targets
  int32_t nch;          // chunks per slice of the histogram and the scatter
  int64_t chunk;        // entries per chunk (the last one may hold fewer)
};

__device__ __forceinline__ int bucket_of(float z, float fcmin, float invw, int nb) {
  const float q = (z - fcmin) * invw;
  return (q < (float)nb) ? (int)q : nb - 1;     // q >= 0; inf / NaN go to the last bucket
}

__device__ __forceinline__ long long fix_a(float v, int eA) {
  return __double2ll_rn(ldexp((double)v, eA));
}

__device__ __forceinline__ long long fix_s(float v, float z, double cmid, int eS) {
  return __double2ll_rn(ldexp((double)v * ((double)z - cmid), eS));
}

// ---------------------------------------------------------------------------
// S1: per (slice, chunk) bucket histogram with fixed-point sums.  Each thread
// loads kHistU projections (and weights) before it touches LDS, so that many
// loads are in flight per wave.
// ---------------------------------------------------------------------------
constexpr int kHistU = 8;

__global__ __launch_bounds__(512) void sort_hist_kernel(SortArgs a) {
  __shared__ uint32_t cnt[2048];
  __shared__ unsigned long long sA[2048], sS[2048];
  const int64_t work = xcd_remap(blockIdx.x, (int64_t)a.nsl * a.nch);
  if (work < 0) return;
  const int p = (int)(work / a.nch), c = (int)(work % a.nch);
  for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
    cnt[b] = 0;
    sA[b] = 0;
    sS[b] = 0;
  }
  __syncthreads();
  const SliceParams sp = a.params[p];
  const int eA = (int)a.misc[1];
  const int64_t l0 = c * a.chunk, l1 = min(a.L, l0 + a.chunk);
  const float *Zp = a.Z + (int64_t)p * a.L;
  for (int64_t lb = l0; lb < l1; lb += 512 * kHistU) {
    float z[kHistU], v[kHistU];
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      const int64_t l = lb + threadIdx.x + 512 * u;
      z[u] = (l < l1) ? Zp[l] : 0.f;
      v[u] = (l < l1 && l >= a.M) ? a.w[l - a.M] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kHistU; ++u) {
      const int64_t l = lb + threadIdx.x + 512 * u;
      if (l < l1) {
        const int b = bucket_of(z[u], sp.fcmin, sp.inv_width, a.nb);
        atomicAdd(&cnt[b], 1u);
        if (l >= a.M) {
          atomicAdd(&sA[b], (unsigned long long)fix_a(v[u], eA));
          atomicAdd(&sS[b], (unsigned long long)fix_s(v[u], z[u], sp.cmid, sp.eS));
        }
      }
    }
  }
  __syncthreads();
  const int64_t base = ((int64_t)p * a.nch + c) * a.nb;
  for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
    a.hcnt[base + b] = cnt[b];
    a.hsum[2 * (base + b)] = (long long)sA[b];
    a.hsum[2 * (base + b) + 1] = (long long)sS[b];
  }
}

// ---------------------------------------------------------------------------
// S2: bucket offsets, chunk offsets, exclusive bucket prefixes (one block per slice)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void sort_scan_kernel(SortArgs a) {
  __shared__ long long sm[64];
  const int p = blockIdx.x;
  const int per = (a.nb + 1023) / 1024;   // buckets per thread (nb <= 2048)
  long long cntv[2] = {0, 0}, Av[2] = {0, 0}, Sv[2] = {0, 0};
  const int64_t base = (int64_t)p * a.nch * a.nb;
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    if (b < a.nb) {
      for (int c = 0; c < a.nch; ++c) {
        const int64_t o = base + (int64_t)c * a.nb + b;
        cntv[q] += a.hcnt[o];
        Av[q] += a.hsum[2 * o];
        Sv[q] += a.hsum[2 * o + 1];
      }
    }
  }
  long long tc, tA, tS;
  long long ec = block_exclusive_scan(cntv[0] + cntv[1], sm, &tc);
  long long eAx = block_exclusive_scan(Av[0] + Av[1], sm, &tA);
  long long eSx = block_exclusive_scan(Sv[0] + Sv[1], sm, &tS);
  uint32_t *boff = a.boff + (int64_t)p * (a.nb + 1);
  long long *bpre = a.bpre + 2 * (int64_t)p * a.nb;
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    if (b < a.nb) {
      boff[b] = (uint32_t)ec;
      bpre[2 * b] = eAx;
      bpre[2 * b + 1] = eSx;
      uint32_t run = (uint32_t)ec;
      for (int c = 0; c < a.nch; ++c) {
        const int64_t o = base + (int64_t)c * a.nb + b;
        const uint32_t v = a.hcnt[o];
        a.hcnt[o] = run;
        run += v;
      }
    }
    ec += cntv[q];
    eAx += Av[q];
    eSx += Sv[q];
  }
  // group descriptors: group g holds the buckets whose start offset lies in
  // [g kSortHalf, (g + 1) kSortHalf); empty groups keep n = 0
  __shared__ uint32_t sboff[2049];
  int4 *desc = a.desc + (int64_t)p * a.G;
  for (int g2 = threadIdx.x; g2 < a.G; g2 += blockDim.x) desc[g2] = make_int4(0, 0, 0, 0);
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    if (b < a.nb) sboff[b] = boff[b];
  }
  if (threadIdx.x == 0) sboff[a.nb] = (uint32_t)a.L;
  __syncthreads();
  for (int q = 0; q < per; ++q) {
    const int b = threadIdx.x * per + q;
    if (b < a.nb) {
      const uint32_t g2 = sboff[b] / kSortHalf;
      const bool first = (b == 0) || (sboff[b - 1] / kSortHalf != g2);
      const bool last = (b == a.nb - 1) || (sboff[b + 1] / kSortHalf != g2);
      if (first) {
        desc[g2].x = b;                  // first bucket
        desc[g2].y = (int)sboff[b];      // first entry
      }
      if (last) {
        desc[g2].z = (int)sboff[b + 1];   // end entry
        desc[g2].w = b;                   // last bucket
      }
    }
  }
  if (threadIdx.x == 0) {
    if (p == 0) *a.fail_count = 0u;
    boff[a.nb] = (uint32_t)a.L;
    a.tot[2 * p] = tA;
    a.tot[2 * p + 1] = tS;
  }
}

// ---------------------------------------------------------------------------
// S3: scatter (key, union index) into buckets.  Each tile of TILE entries is
// first ordered by bucket in LDS, so the global writes come as runs of
// consecutive positions per bucket instead of isolated 8-byte stores.  The next
// tile's projections are loaded while the current one is processed, the keys
// stay in registers until they are placed, and the tile counters alternate
// between two arrays, so a tile takes four barriers plus the one of its scan.
// Tiles of 12288 entries (152 KB of LDS) give longer runs than tiles of 8192;
// the launch takes whichever cuts a chunk into fewer tiles, the smaller on a tie
// (a nearly empty last tile costs as many barriers as a full one).
// ---------------------------------------------------------------------------
constexpr int kScatThreads = 1024;

template <int TILE>
__global__ __launch_bounds__(kScatThreads) void sort_scatter_kernel(SortArgs a) {
  constexpr int kScatTile = TILE;
  constexpr int kScatPer = kScatTile / kScatThreads;
  __shared__ unsigned long long tk[kScatTile];
  __shared__ uint16_t tb[kScatTile];
  __shared__ uint32_t cursor[2048], tcnt[2][2048], tstart[2048];
  __shared__ uint32_t red[kScatThreads / 64];
  const int64_t work = xcd_remap(blockIdx.x, (int64_t)a.nsl * a.nch);
  if (work < 0) return;
  const int p = (int)(work / a.nch), c = (int)(work % a.nch);
  const int64_t base = ((int64_t)p * a.nch + c) * a.nb;
  for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
    cursor[b] = a.hcnt[base + b];
    tcnt[0][b] = 0;
    tcnt[1][b] = 0;
  }
  const SliceParams sp = a.params[p];
  const int64_t l0 = c * a.chunk, l1 = min(a.L, l0 + a.chunk);
  const float *Zp = a.Z + (int64_t)p * a.L;
  unsigned long long *kp = a.keys + (int64_t)p * a.L;
  const int per = (a.nb + kScatThreads - 1) / kScatThreads;    // buckets per thread in the scan
  float zn[kScatPer];
#pragma unroll
  for (int q = 0; q < kScatPer; ++q) {
    const int64_t l = l0 + threadIdx.x + q * kScatThreads;
    zn[q] = (l < l1) ? Zp[l] : 0.f;
  }
  __syncthreads();
  int buf = 0;
  for (int64_t t0 = l0; t0 < l1; t0 += kScatTile, buf ^= 1) {
    const int tn = (int)min((int64_t)kScatTile, l1 - t0);
    float zc[kScatPer];
#pragma unroll
    for (int q = 0; q < kScatPer; ++q) zc[q] = zn[q];
    if (t0 + kScatTile < l1) {
#pragma unroll
      for (int q = 0; q < kScatPer; ++q) {
        const int64_t l = t0 + kScatTile + threadIdx.x + q * kScatThreads;
        zn[q] = (l < l1) ? Zp[l] : 0.f;
      }
    }
    uint32_t *cntb = tcnt[buf];
    // bucket of every entry of the tile; ranks within its bucket
    int bk[kScatPer];
    uint32_t rk[kScatPer];
    unsigned long long kv[kScatPer];
#pragma unroll
    for (int q = 0; q < kScatPer; ++q) {
      const int i = threadIdx.x + q * kScatThreads;
      bk[q] = 0;
      rk[q] = 0;
      kv[q] = 0;
      if (i < tn) {
        bk[q] = bucket_of(zc[q], sp.fcmin, sp.inv_width, a.nb);
        rk[q] = atomicAdd(&cntb[bk[q]], 1u);
        kv[q] = (unsigned long long)float_key(zc[q]) | ((unsigned long long)(uint32_t)(t0 + i) << 32);
      }
    }
    __syncthreads();
    // exclusive scan of the tile's bucket counts
    uint32_t loc = 0;
    for (int q = 0; q < per; ++q) {
      const int b = threadIdx.x * per + q;
      if (b < a.nb) loc += cntb[b];
    }
    uint32_t tot;
    uint32_t ex = block_excl_sum<kScatThreads / 64>(loc, red, &tot);
    for (int q = 0; q < per; ++q) {
      const int b = threadIdx.x * per + q;
      if (b < a.nb) {
        tstart[b] = ex;
        ex += cntb[b];
      }
    }
    __syncthreads();
    // place the tile in bucket order in LDS (entries of one bucket stay in tile order)
#pragma unroll
    for (int q = 0; q < kScatPer; ++q) {
      const int i = threadIdx.x + q * kScatThreads;
      if (i < tn) {
        const uint32_t pos = tstart[bk[q]] + rk[q];
        tk[pos] = kv[q];
        tb[pos] = (uint16_t)bk[q];
      }
    }
    __syncthreads();
    // consecutive LDS entries -> consecutive global positions within a bucket
    for (int i = threadIdx.x; i < tn; i += blockDim.x) {
      const int b = tb[i];
      kp[cursor[b] + (uint32_t)i - tstart[b]] = tk[i];
    }
    __syncthreads();
    // the next tile counts into the other array; this one is cleared for the tile after
    for (int b = threadIdx.x; b < a.nb; b += blockDim.x) {
      cursor[b] += cntb[b];
      cntb[b] = 0;
    }
  }
}

// ---------------------------------------------------------------------------
// S4 helpers: stable ranking of a tile of <= kSortCap LDS entries by an 8-bit digit
// ---------------------------------------------------------------------------
constexpr int kR = kSortCap / 256;   // rounds of 64 per wave (16)

struct RankState {
  uint32_t hw[4][256];     // per-wave digit counts, then per-wave digit offsets
  long long sm[64];
  uint32_t flag;
};

constexpr int kNS = 2048;            // value-linear sub-buckets of a group sorted in LDS
constexpr int kSubRunMax = 64;       // longest sub-bucket run sorted by insertion

// Ranks entries [0, n) of (kin, iin) by digit(d) and returns, in pos[r] for the
// entries this thread owns (position (wid * kR + r) * 64 + lane), their offset
// within the tile's stable counting-sort order.  If tile_tot is given it
// receives the per-digit totals (before return, synchronised).
template <typename DigitFn>
__device__ __forceinline__ void rank_tile(const uint32_t *kin, const uint32_t *iin, int n, DigitFn digit,
                                          RankState &st, int (&pos)[kR], uint32_t (&dg)[kR],
                                          uint32_t *tile_tot) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < 4 * 256; i += 256) (&st.hw[0][0])[i] = 0;
  __syncthreads();
  const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = (wid * kR + r) * 64 + lane;
    const bool valid = i < n;
    const uint32_t d = valid ? digit(kin[i], iin[i]) : 0u;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const unsigned long long bm = __ballot(valid && ((d >> bit) & 1u));
      peers &= ((d >> bit) & 1u) ? bm : ~bm;
    }
    int rank = 0;
    if (valid) {
      const uint32_t old = st.hw[wid][d];
      rank = (int)old + __popcll(peers & lt);
      if ((peers & lt) == 0ull) st.hw[wid][d] = old + (uint32_t)__popcll(peers);
    }
    pos[r] = rank;
    dg[r] = d;
  }
  __syncthreads();
  {
    const int d = threadIdx.x;   // 256 threads = 256 digits
    const uint32_t c0 = st.hw[0][d], c1 = st.hw[1][d], c2 = st.hw[2][d], c3 = st.hw[3][d];
    const long long tot = (long long)c0 + c1 + c2 + c3;
    long long all;
    const long long base = block_exclusive_scan(tot, st.sm, &all);
    if (tile_tot) tile_tot[d] = (uint32_t)tot;
    st.hw[0][d] = (uint32_t)base;
    st.hw[1][d] = (uint32_t)(base + c0);
    st.hw[2][d] = (uint32_t)(base + c0 + c1);
    st.hw[3][d] = (uint32_t)(base + c0 + c1 + c2);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = (wid * kR + r) * 64 + lane;
    if (i < n) pos[r] += (int)st.hw[wid][dg[r]];
  }
}

struct GroupShared {
  uint32_t K[2][kSortCap];
  uint32_t I[2][kSortCap];
  RankState rs;
  uint32_t gbase[256], grun[256], ttot[256];
  uint32_t red[8];
};

// One stable counting-sort pass inside LDS: (K[src], I[src]) -> (K[src^1], I[src^1]).
template <typename DigitFn>
__device__ __forceinline__ void lds_pass(GroupShared &g, int src, int n, DigitFn digit) {
  int pos[kR];
  uint32_t dg[kR];
  rank_tile(g.K[src], g.I[src], n, digit, g.rs, pos, dg, nullptr);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t kk[kR], ii[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = (wid * kR + r) * 64 + lane;
    if (i < n) {
      kk[r] = g.K[src][i];
      ii[r] = g.I[src][i];
    }
  }
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    const int i = (wid * kR + r) * 64 + lane;
    if (i < n) {
      g.K[src ^ 1][pos[r]] = kk[r];
      g.I[src ^ 1][pos[r]] = ii[r];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ int bitlen(uint32_t v) { return v ? 32 - __clz((int)v) : 0; }

// block-wide min / max of n LDS values
__device__ __forceinline__ void block_minmax(const uint32_t *v, int n, uint32_t *red, uint32_t &mn,
                                             uint32_t &mx) {
  uint32_t lo = 0xffffffffu, hi = 0u;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    lo = min(lo, v[i]);
    hi = max(hi, v[i]);
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    red[wid] = lo;
    red[4 + wid] = hi;
  }
  __syncthreads();
  mn = min(min(red[0], red[1]), min(red[2], red[3]));
  mx = max(max(red[4], red[5]), max(red[6], red[7]));
  __syncthreads();
}

// LDS index of entry i in a padded array: one spare word after every 16 entries,
// so 16 consecutive entries per thread sit at a stride of 17 words across lanes.
__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }
__device__ __forceinline__ int nopad(int i) { return i; }

// Fixed-point prefix scan over the sorted tile [0, n) with carry-in (cA, cS);
// emits t at the targets and the permutation; adds the tile totals to (cA, cS).
// Thread t owns the 16 consecutive entries [16t, 16t+16): a serial prefix in
// registers plus one block scan of the per-thread totals.  IX maps an entry to
// its LDS index (padded arrays avoid bank conflicts).
template <int (*IX)(int)>
__device__ __forceinline__ void scan_emit(const SortArgs &a, int p, const SliceParams &sp, int eA,
                                          const uint32_t *K, const uint32_t *I, const float *W, int n,
                                          int64_t out_pos, long long &cA, long long &cS, long long Atot,
                                          long long Stot, long long *sm) {
  constexpr int per = kSortCap / 256;   // 16 consecutive entries per thread
  const int i0 = threadIdx.x * per;
  long long fa[per], fs[per];
  long long lA = 0, lS = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int i = i0 + q;
    fa[q] = 0;
    fs[q] = 0;
    if (i < n) {
      const uint32_t idx = I[IX(i)];
      if ((int64_t)idx >= a.M) {
        const float v = W ? W[IX(i)] : a.w[idx - a.M];
        fa[q] = fix_a(v, eA);
        fs[q] = fix_s(v, key_float(K[IX(i)]), sp.cmid, sp.eS);
      }
    }
    lA += fa[q];
    lS += fs[q];
  }
  long long totA, totS;
  long long exA = block_exclusive_scan(lA, sm, &totA) + cA;
  long long exS = block_exclusive_scan(lS, sm, &totS) + cS;
  const double sa = ldexp(1.0, -eA), ss = ldexp(1.0, -sp.eS);
  float *tp = a.t + (int64_t)p * a.M;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int i = i0 + q;
    if (i < n) {
      const uint32_t idx = I[IX(i)];
      if ((int64_t)idx < a.M) {
        const double zb = (double)key_float(K[IX(i)]) - sp.cmid;
        const long long dA = 2 * exA - Atot;
        const long long dS = 2 * exS - Stot;
        tp[idx] = (float)(-a.cneg * (zb * ((double)dA * sa) - (double)dS * ss));
      }
      if (a.perm) a.perm[(int64_t)p * a.L + out_pos + i] = (int32_t)idx;
    }
    exA += fa[q];
    exS += fs[q];
  }
  cA += totA;
  cS += totS;
}

// Derivative emission (see the top of the file) for a group sorted in LDS: the
// exclusive fixed-point prefixes of the weights go to the free LDS buffers (low and
// high 32 bits), and the end of each target's run of equal keys is found by binary
// search in the sorted keys; D = -c' (E_i + E_end - A_tot).
__device__ void deriv_emit_lds(const SortArgs &a, int p, int eA, const uint32_t *K, const uint32_t *I,
                               uint32_t *Elo, uint32_t *Ehi, int n, int64_t out_pos, long long cA, long long Atot,
                               long long *sm) {
  constexpr int per = kSortCap / 256;
  const int i0 = threadIdx.x * per;
  long long fa[per];
  long long lA = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int i = i0 + q;
    fa[q] = (i < n && (int64_t)I[i] >= a.M) ? fix_a(a.w[I[i] - a.M], eA) : 0;
    lA += fa[q];
  }
  long long tot;
  long long ex = block_exclusive_scan(lA, sm, &tot) + cA;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int i = i0 + q;
    if (i < n) {
      Elo[i] = (uint32_t)ex;
      Ehi[i] = (uint32_t)((unsigned long long)ex >> 32);
    }
    ex += fa[q];
  }
  __syncthreads();
  const long long endA = cA + tot;
  const double sa = ldexp(1.0, -eA);
  float *tp = a.t + (int64_t)p * a.M;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t idx = I[i];
    if (a.perm) a.perm[(int64_t)p * a.L + out_pos + i] = (int32_t)idx;
    if ((int64_t)idx < a.M) {
      const uint32_t k = K[i];
      int lo = i + 1, hi = n;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (K[mid] <= k) lo = mid + 1; else hi = mid;
      }
      const long long Ei = (long long)(((unsigned long long)Ehi[i] << 32) | Elo[i]);
      const long long Eb = (lo < n) ? (long long)(((unsigned long long)Ehi[lo] << 32) | Elo[lo]) : endA;
      tp[idx] = (float)(-a.cneg * ((double)(Ei + Eb - Atot) * sa));
    }
  }
  __syncthreads();
}

// The same for a large group sorted in global memory (src, n entries): the prefixes
// go to the free buffer dst in a first pass over LDS tiles.
__device__ void deriv_emit_stream(const SortArgs &a, GroupShared &g, int p, int eA,
                                  const unsigned long long *src, unsigned long long *dst, int64_t n,
                                  int64_t out_pos, long long cA, long long Atot) {
  constexpr int per = kSortCap / 256;
  long long *E = reinterpret_cast<long long *>(dst);
  long long carry = cA;
  for (int64_t t0 = 0; t0 < n; t0 += kSortCap) {
    const int tn = (int)min((int64_t)kSortCap, n - t0);
    const int i0 = threadIdx.x * per;
    long long fa[per];
    long long lA = 0;
#pragma unroll
    for (int q = 0; q < per; ++q) {
      const int i = i0 + q;
      fa[q] = 0;
      if (i < tn) {
        const uint32_t idx = (uint32_t)(src[t0 + i] >> 32);
        if ((int64_t)idx >= a.M) fa[q] = fix_a(a.w[idx - a.M], eA);
      }
      lA += fa[q];
    }
    long long tot;
    long long ex = block_exclusive_scan(lA, g.rs.sm, &tot) + carry;
#pragma unroll
    for (int q = 0; q < per; ++q) {
      const int i = i0 + q;
      if (i < tn) E[t0 + i] = ex;
      ex += fa[q];
    }
    carry += tot;
    __syncthreads();
  }
  const long long endA = carry;
  const double sa = ldexp(1.0, -eA);
  float *tp = a.t + (int64_t)p * a.M;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const unsigned long long e = src[i];
    const uint32_t idx = (uint32_t)(e >> 32);
    if (a.perm) a.perm[(int64_t)p * a.L + out_pos + i] = (int32_t)idx;
    if ((int64_t)idx < a.M) {
      const uint32_t k = (uint32_t)e;
      int64_t lo = i + 1, hi = n;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((uint32_t)src[mid] <= k) lo = mid + 1; else hi = mid;
      }
      const long long Eb = (lo < n) ? E[lo] : endA;
      tp[idx] = (float)(-a.cneg * ((double)(E[i] + Eb - Atot) * sa));
    }
  }
  __syncthreads();
}

// Sort the tile's equal-key runs by union index.  Returns false if a run is
// longer than 32 (then the caller re-sorts the whole tile by (key, index)).
__device__ __forceinline__ bool fix_ties(uint32_t *K, uint32_t *I, int n, uint32_t *flag) {
  if (threadIdx.x == 0) *flag = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const bool head = (i == 0) || (K[i] != K[i - 1]);
    if (head && i + 1 < n && K[i + 1] == K[i]) {
      int e = i + 1;
      while (e < n && K[e] == K[i] && e - i <= 32) ++e;
      if (e - i > 32) {
        *flag = 1;
      } else {
        for (int a2 = i + 1; a2 < e; ++a2) {      // insertion sort of I[i..e)
          const uint32_t v = I[a2];
          int b = a2 - 1;
          while (b >= i && I[b] > v) {
            I[b + 1] = I[b];
            --b;
          }
          I[b + 1] = v;
        }
      }
    }
  }
  __syncthreads();
  const bool ok = (*flag == 0);
  __syncthreads();
  return ok;
}

// Streaming stable LSD pass over a segment of global memory (one workgroup).
template <typename DigitFn>
__device__ void stream_pass(GroupShared &g, const unsigned long long *src, unsigned long long *dst, int64_t n,
                            DigitFn digit) {
  // global digit histogram
  for (int i = threadIdx.x; i < 256; i += 256) g.gbase[i] = 0;
  __syncthreads();
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const unsigned long long e = src[i];
    atomicAdd(&g.gbase[digit((uint32_t)e, (uint32_t)(e >> 32))], 1u);
  }
  __syncthreads();
  {
    long long all;
    const long long v = g.gbase[threadIdx.x];
    const long long ex = block_exclusive_scan(v, g.rs.sm, &all);
    g.gbase[threadIdx.x] = (uint32_t)ex;
    g.grun[threadIdx.x] = 0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t t0 = 0; t0 < n; t0 += kSortCap) {
    const int tn = (int)min((int64_t)kSortCap, n - t0);
    for (int i = threadIdx.x; i < tn; i += 256) {
      const unsigned long long e = src[t0 + i];
      g.K[0][i] = (uint32_t)e;
      g.I[0][i] = (uint32_t)(e >> 32);
    }
    __syncthreads();
    int pos[kR];
    uint32_t dg[kR];
    rank_tile(g.K[0], g.I[0], tn, digit, g.rs, pos, dg, g.ttot);
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int i = (wid * kR + r) * 64 + lane;
      if (i < tn) {
        const uint32_t d = dg[r];
        const int within = pos[r] - (int)g.rs.hw[0][d];      // offset among this tile's digit-d entries
        const int64_t o = (int64_t)g.gbase[d] + g.grun[d] + within;
        dst[o] = (unsigned long long)g.K[0][i] | ((unsigned long long)g.I[0][i] << 32);
      }
    }
    __syncthreads();
    g.grun[threadIdx.x] += g.ttot[threadIdx.x];
    __syncthreads();
  }
}

// Locates work item (slice, group): the buckets b whose start offset lies in
// [group * kSortHalf, (group + 1) * kSortHalf), i.e. whole consecutive buckets.
struct GroupDesc {
  int p, b_lo, b_hi;
  int64_t e_lo;
  int n;
};

__device__ __forceinline__ GroupDesc group_desc(const SortArgs &a, int64_t item) {
  const int4 v = a.desc[item];
  GroupDesc d;
  d.p = (int)(item / a.G);
  d.b_lo = v.x;
  d.b_hi = v.w;
  d.e_lo = v.y;
  d.n = v.z - v.y;
  return d;
}

// Radix / streaming sort of one group the fast kernel handed over.
__device__ void fallback_group(const SortArgs &a, GroupShared &g, int64_t item) {
  const GroupDesc dsc = group_desc(a, item);
  const int p = dsc.p;
  const int b_lo = dsc.b_lo;
  const int64_t e_lo = dsc.e_lo;
  const int64_t n = dsc.n;
  if (n <= 0) return;
  const SliceParams sp = a.params[p];
  const int eA = (int)a.misc[1];
  long long cA = a.bpre[2 * ((int64_t)p * a.nb + b_lo)];
  long long cS = a.bpre[2 * ((int64_t)p * a.nb + b_lo) + 1];
  const long long Atot = a.tot[2 * p], Stot = a.tot[2 * p + 1];
  unsigned long long *seg = a.keys + (int64_t)p * a.L + e_lo;

  if (n <= kSortCap) {
    const int nn = (int)n;
    for (int i = threadIdx.x; i < nn; i += 256) {
      const unsigned long long e = seg[i];
      g.K[0][i] = (uint32_t)e;
      g.I[0][i] = (uint32_t)(e >> 32);
    }
    __syncthreads();
    uint32_t kmin, kmax;
    block_minmax(g.K[0], nn, g.red, kmin, kmax);
    const int kbits = bitlen(kmax - kmin);
    int cur = 0;
    for (int sh = 0; sh < kbits; sh += 8) {
      lds_pass(g, cur, nn, [=](uint32_t k, uint32_t) { return ((k - kmin) >> sh) & 255u; });
      cur ^= 1;
    }
    if (!fix_ties(g.K[cur], g.I[cur], nn, &g.rs.flag)) {
      // long runs of equal keys: stable sort by index, then by key
      uint32_t imin, imax;
      block_minmax(g.I[cur], nn, g.red, imin, imax);
      const int ibits = bitlen(imax - imin);
      for (int sh = 0; sh < ibits; sh += 8) {
        lds_pass(g, cur, nn, [=](uint32_t, uint32_t i) { return ((i - imin) >> sh) & 255u; });
        cur ^= 1;
      }
      for (int sh = 0; sh < kbits; sh += 8) {
        lds_pass(g, cur, nn, [=](uint32_t k, uint32_t) { return ((k - kmin) >> sh) & 255u; });
        cur ^= 1;
      }
    }
    if (a.deriv)
      deriv_emit_lds(a, p, eA, g.K[cur], g.I[cur], g.K[cur ^ 1], g.I[cur ^ 1], nn, e_lo, cA, Atot, g.rs.sm);
    else
      scan_emit<nopad>(a, p, sp, eA, g.K[cur], g.I[cur], nullptr, nn, e_lo, cA, cS, Atot, Stot, g.rs.sm);
    return;
  }

  // Large group: stable LSD radix sort by (key, index) streaming through global memory.
  unsigned long long *seg2 = a.keys2 + (int64_t)p * a.L + e_lo;
  uint32_t kmin = 0xffffffffu, kmax = 0u, imin = 0xffffffffu, imax = 0u;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const unsigned long long e = seg[i];
    kmin = min(kmin, (uint32_t)e);
    kmax = max(kmax, (uint32_t)e);
    imin = min(imin, (uint32_t)(e >> 32));
    imax = max(imax, (uint32_t)(e >> 32));
  }
  {
    // reduce the four values across the block through LDS
    for (int off = 32; off > 0; off >>= 1) {
      kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, off, 64));
      kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, off, 64));
      imin = min(imin, (uint32_t)__shfl_xor((int)imin, off, 64));
      imax = max(imax, (uint32_t)__shfl_xor((int)imax, off, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      g.rs.hw[0][wid] = kmin;
      g.rs.hw[1][wid] = kmax;
      g.rs.hw[2][wid] = imin;
      g.rs.hw[3][wid] = imax;
    }
    __syncthreads();
    kmin = min(min(g.rs.hw[0][0], g.rs.hw[0][1]), min(g.rs.hw[0][2], g.rs.hw[0][3]));
    kmax = max(max(g.rs.hw[1][0], g.rs.hw[1][1]), max(g.rs.hw[1][2], g.rs.hw[1][3]));
    imin = min(min(g.rs.hw[2][0], g.rs.hw[2][1]), min(g.rs.hw[2][2], g.rs.hw[2][3]));
    imax = max(max(g.rs.hw[3][0], g.rs.hw[3][1]), max(g.rs.hw[3][2], g.rs.hw[3][3]));
    __syncthreads();
  }
  const int kbits = bitlen(kmax - kmin), ibits = bitlen(imax - imin);
  unsigned long long *src = seg, *dst = seg2;
  for (int sh = 0; sh < ibits; sh += 8) {
    stream_pass(g, src, dst, n, [=](uint32_t, uint32_t i) { return ((i - imin) >> sh) & 255u; });
    unsigned long long *tmp = src; src = dst; dst = tmp;
  }
  for (int sh = 0; sh < kbits; sh += 8) {
    stream_pass(g, src, dst, n, [=](uint32_t k, uint32_t) { return ((k - kmin) >> sh) & 255u; });
    unsigned long long *tmp = src; src = dst; dst = tmp;
  }
  if (a.deriv) {
    deriv_emit_stream(a, g, p, eA, src, dst, n, e_lo, cA, Atot);
    return;
  }
  for (int64_t t0 = 0; t0 < n; t0 += kSortCap) {
    const int tn = (int)min((int64_t)kSortCap, n - t0);
    for (int i = threadIdx.x; i < tn; i += 256) {
      const unsigned long long e = src[t0 + i];
      g.K[0][i] = (uint32_t)e;
      g.I[0][i] = (uint32_t)(e >> 32);
    }
    __syncthreads();
    scan_emit<nopad>(a, p, sp, eA, g.K[0], g.I[0], nullptr, tn, e_lo + t0, cA, cS, Atot, Stot, g.rs.sm);
    __syncthreads();
  }
}


__global__ __launch_bounds__(256) void sort_fallback_kernel(SortArgs a) {
  __shared__ GroupShared g;
  const uint32_t count = *a.fail_count;
  for (uint32_t j = blockIdx.x; j < count; j += gridDim.x) {
    fallback_group(a, g, a.fail_list[j]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// S4 fast path.  A group (<= kSortCap entries) is sorted by (key, index) with
// one counting pass into kNS value-linear sub-buckets over [min, max] of the
// group (a monotone map); inside a sub-bucket every entry counts the entries
// smaller than itself and moves to that rank.  The keys stay in registers until
// they are scattered into sub-bucket order in LDS, the weights are gathered up
// front and carried along, and the next group's keys are loaded while the
// current group is processed.  Groups that are too large, have all keys equal
// or a sub-bucket longer than kSubRunMax go to the fallback list.
// 512 threads, kFPer = 8 consecutive entries per thread in the scan.
// ---------------------------------------------------------------------------
constexpr int kFThreads = 512;
constexpr int kFPer = kSortCap / kFThreads;          // 8
constexpr int kFWaves = kFThreads / 64;
constexpr int kFCapPad = kSortCap + kSortCap / 8;    // pad8 layout

// one spare word per 8 entries (stride 9 words between threads' 8-entry blocks)
__device__ __forceinline__ int pad8(int i) { return i + (i >> 3); }
// one spare word per 4 counters (stride 5 words between threads' 4-counter blocks)
__device__ __forceinline__ int pad4(int i) { return i + (i >> 2); }

struct FastShared {
  uint32_t K[kFCapPad];
  uint32_t I[kFCapPad];
  float W[kFCapPad];
  uint16_t inv[kFCapPad];      // sorted position -> entry (pad8 layout)
  uint32_t cnt[kNS + kNS / 4];
  double pr[2 * kFWaves];      // wave totals of the (A, S) prefix scan
  uint32_t cr[kFWaves];        // wave totals of the counter scan
  uint32_t flag;
};

// The keys are read once, so they are loaded non-temporally: they then do not push
// out of L2 the lines of t that the slice's other groups have yet to fill in
// (t is written by target index, a few values per line per group).
__device__ __forceinline__ void load_group_keys(const SortArgs &a, const GroupDesc &d,
                                                unsigned long long (&kr)[kFPer]) {
  const unsigned long long *seg = a.keys + (int64_t)d.p * a.L + d.e_lo;
#pragma unroll
  for (int q = 0; q < kFPer; ++q) {
    const int i = threadIdx.x + kFThreads * q;
    kr[q] = (d.n <= kSortCap && i < d.n) ? __builtin_nontemporal_load(seg + i) : ~0ull;
  }
}

__device__ __forceinline__ void push_fallback(const SortArgs &a, int64_t item) {
  if (threadIdx.x == 0) a.fail_list[atomicAdd(a.fail_count, 1u)] = (uint32_t)item;
}

// Sub-bucket of a key within its group: the group's buckets [b_lo, b_hi] cut into kNS
// equal parts of the bucket coordinate q = (z - c_min) w, the same FP32 expression
// that put the key in its bucket (so q >= b_lo).  A monotone map of the key, so
// sub-bucket order is value order.
struct SubMap {
  float fcmin, invw, qlo, scale;
};

__device__ __forceinline__ int sub_bucket(uint32_t key, const SubMap &m) {
  const float q = (key_float(key) - m.fcmin) * m.invw;
  const float s = (q - m.qlo) * m.scale;
  return (s < (float)kNS) ? (int)s : kNS - 1;
}

// Per-group scalars the scan needs (bucket prefixes, slice totals, slice
// parameters), loaded when the group starts so their latency overlaps the sort.
struct GroupScalars {
  long long preA, preS, totA, totS;
  double cmid;
  int eS;
  SubMap sub;
};

__device__ __forceinline__ GroupScalars group_scalars(const SortArgs &a, const GroupDesc &d) {
  GroupScalars s;
  const int64_t o = 2 * ((int64_t)d.p * a.nb + d.b_lo);
  s.preA = a.bpre[o];
  s.preS = a.bpre[o + 1];
  s.totA = a.tot[2 * d.p];
  s.totS = a.tot[2 * d.p + 1];
  s.cmid = a.params[d.p].cmid;
  s.eS = a.params[d.p].eS;
  s.sub.fcmin = a.params[d.p].fcmin;
  s.sub.invw = a.params[d.p].inv_width;
  s.sub.qlo = (float)d.b_lo;
  s.sub.scale = (float)kNS / (float)(d.b_hi - d.b_lo + 1);
  return s;
}

// Scan of a sorted group: FP64 prefix sums inside the group, taken in its
// canonical (key, index) order (so the rounding is the same on every run), on
// top of the exact fixed-point prefix of the group's first bucket.  W holds the
// weights of the sources (0 for targets).  Thread t owns the sorted positions
// [per t, per (t + 1)) with per = ceil(n / threads), so that every wave takes part
// however large the group; its entries stay in registers from the prefix pass to the
// output pass.  In derivative mode a target also adds the sources
// tied with it: the rest of its run of equal keys (targets precede tied sources
// in the (key, index) order, and a run never crosses a bucket).
template <bool DERIV>
__device__ __forceinline__ void scan_emit_fast(const SortArgs &a, int p, const GroupScalars &gs, int eA,
                                               FastShared &f, int n, int64_t out_pos) {
  const int per = (n + kFThreads - 1) / kFThreads;   // <= kFPer
  const int i0 = threadIdx.x * per;
  double lA = 0.0, lS = 0.0;
  uint32_t kq[kFPer], iq[kFPer];
  float wq[kFPer];
#pragma unroll
  for (int q = 0; q < kFPer; ++q) {
    const int j = i0 + q;
    kq[q] = 0;
    iq[q] = 0;
    wq[q] = 0.f;
    if (q < per && j < n) {
      const int e = pad8(f.inv[pad8(j)]);
      kq[q] = f.K[e];
      iq[q] = f.I[e];
      wq[q] = f.W[e];
      const double v = (double)wq[q];
      lA += v;
      lS += v * ((double)key_float(kq[q]) - gs.cmid);
    }
  }
  double gA, gS;
  block_excl_sum2<kFWaves>(lA, lS, f.pr, &gA, &gS);
  const double sa = ldexp(1.0, -eA), ss = ldexp(1.0, -gs.eS);
  double exA = lA + (double)gs.preA * sa, exS = lS + (double)gs.preS * ss;
  const double totAd = (double)gs.totA * sa, totSd = (double)gs.totS * ss;
  float *tp = a.t + (int64_t)p * a.M;
#pragma unroll
  for (int q = 0; q < kFPer; ++q) {
    const int j = i0 + q;
    if (q < per && j < n) {
      const uint32_t kk = kq[q], ii = iq[q];
      const double v = (double)wq[q];
      const double zb = (double)key_float(kk) - gs.cmid;
      if ((int64_t)ii < a.M) {
        if (DERIV) {
          double eq = 0.0;
          for (int j2 = j + 1; j2 < n; ++j2) {
            const int e2 = pad8(f.inv[pad8(j2)]);
            if (f.K[e2] != kk) break;
            eq += (double)f.W[e2];
          }
          tp[ii] = (float)(-a.cneg * (2.0 * exA + eq - totAd));
        } else {
          tp[ii] = (float)(-a.cneg * (zb * (2.0 * exA - totAd) - (2.0 * exS - totSd)));
        }
      }
      if (a.perm) a.perm[(int64_t)p * a.L + out_pos + j] = (int32_t)ii;
      exA += v;
      exS += v * zb;
    }
  }
}

template <bool DERIV>
__global__ __launch_bounds__(kFThreads, 4) void sort_fast_kernel(SortArgs a) {
  __shared__ FastShared f;
  const int64_t total = (int64_t)a.nsl * a.G;
  // XCD-contiguous ranges of work items; the blocks of an XCD stride through it
  const int x = blockIdx.x & 7, r = blockIdx.x >> 3, gx = gridDim.x >> 3;
  const int64_t per_x = (total + 7) / 8;
  const int64_t lo = x * per_x, hi = min(total, lo + per_x);
  int64_t item = lo + r;
  // descriptors run two items ahead of the keys, the keys one item ahead of the sort
  GroupDesc nd{}, nd2{};
  unsigned long long nk[kFPer];
  if (item < hi) {
    nd = group_desc(a, item);
    load_group_keys(a, nd, nk);
  }
  if (item + gx < hi) nd2 = group_desc(a, item + gx);
  const int eA = (int)a.misc[1];
  // the first group's counters are cleared here, every later group's at the end of the
  // group before it (the flag likewise)
  for (int i = threadIdx.x; i < kNS + kNS / 4; i += kFThreads) f.cnt[i] = 0;
  if (threadIdx.x == 0) f.flag = 0;
  __syncthreads();
  while (item < hi) {
    const GroupDesc d = nd;
    unsigned long long kc[kFPer];
#pragma unroll
    for (int q = 0; q < kFPer; ++q) kc[q] = nk[q];
    const int64_t next = item + gx;
    if (next < hi) {
      nd = nd2;
      load_group_keys(a, nd, nk);
      if (next + gx < hi) nd2 = group_desc(a, next + gx);
    }
    const int64_t cur_item = item;
    item = next;
    if (d.n <= 0) continue;
    if (d.n > kSortCap) {
      push_fallback(a, cur_item);
      continue;
    }
    const int n = d.n, p = d.p;
    const GroupScalars gs = group_scalars(a, d);
    // weights of the sources, gathered now and used at the scatter
    float wv[kFPer];
#pragma unroll
    for (int q = 0; q < kFPer; ++q) {
      const uint32_t idx = (uint32_t)(kc[q] >> 32);
      wv[q] = (threadIdx.x + kFThreads * q < n && (int64_t)idx >= a.M) ? a.w[idx - a.M] : 0.f;
    }
    int sb[kFPer];
#pragma unroll
    for (int q = 0; q < kFPer; ++q) {
      sb[q] = sub_bucket((uint32_t)kc[q], gs.sub);
      if (threadIdx.x + kFThreads * q < n) atomicAdd(&f.cnt[pad4(sb[q])], 1u);
    }
    __syncthreads();
    {
      // exclusive scan of the counters, 4 consecutive per thread (stride 5 words)
      constexpr int per = kNS / kFThreads;
      uint32_t loc[per];
      uint32_t sum = 0;
#pragma unroll
      for (int q = 0; q < per; ++q) {
        loc[q] = f.cnt[pad4(threadIdx.x * per + q)];
        sum += loc[q];
      }
      uint32_t tot;
      uint32_t ex = block_excl_sum<kFWaves>(sum, f.cr, &tot);
#pragma unroll
      for (int q = 0; q < per; ++q) {
        f.cnt[pad4(threadIdx.x * per + q)] = ex;
        ex += loc[q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kFPer; ++q) {
      if (threadIdx.x + kFThreads * q < n) {
        const int pos = pad8((int)atomicAdd(&f.cnt[pad4(sb[q])], 1u));
        f.K[pos] = (uint32_t)kc[q];
        f.I[pos] = (uint32_t)(kc[q] >> 32);
        f.W[pos] = wv[q];
      }
    }
    __syncthreads();
    // cnt[sb] is now the end of sub-bucket sb.  Rank every entry inside its run by
    // (key, index) -- independent LDS reads, no serial chain -- and record which
    // entry lands at each sorted position.
#pragma unroll
    for (int q = 0; q < kFPer; ++q) {
      const int i = threadIdx.x + kFThreads * q;
      if (i < n) {
        const uint32_t kk = f.K[pad8(i)], ii = f.I[pad8(i)];
        const int s = sub_bucket(kk, gs.sub);
        const int e = (int)f.cnt[pad4(s)];
        const int b = s ? (int)f.cnt[pad4(s - 1)] : 0;
        int rank = 0;
        if (e - b > kSubRunMax) {
          f.flag = 1;
        } else {
          const unsigned long long v = ((unsigned long long)kk << 32) | ii;
          for (int j = b; j < e; ++j)
            rank += ((((unsigned long long)f.K[pad8(j)] << 32) | f.I[pad8(j)]) < v) ? 1 : 0;
        }
        f.inv[pad8(min(b + rank, kSortCap - 1))] = (uint16_t)i;
      }
    }
    __syncthreads();
    // a run too long to rank (equal or tightly clustered keys) hands the group over
    const bool handed_over = f.flag != 0;
    // the counters are not read again in this group: clear them for the next one
    for (int i = threadIdx.x; i < kNS + kNS / 4; i += kFThreads) f.cnt[i] = 0;
    if (handed_over)
      push_fallback(a, cur_item);
    else
      scan_emit_fast<DERIV>(a, p, gs, eA, f, n, d.e_lo);
    __syncthreads();
    if (threadIdx.x == 0) f.flag = 0;
  }
}

hipError_t launch_sort_path(const ExecArgs &a) {
  const ksum_plan &pl = *a.plan;
  const Layout &lay = *a.lay;
  SortArgs s{};
  s.nsl = a.nsl;
  s.nb = lay.nb;
  s.G = lay.sort_groups;
  s.L = lay.L;
  s.M = lay.M;
  s.Z = wsp<float>(a, lay.off_z);
  s.w = a.w;
  s.params = wsp<SliceParams>(a, lay.off_params);
  s.misc = wsp<double>(a, lay.off_misc);
  s.hcnt = wsp<uint32_t>(a, lay.off_hcnt);
  s.hsum = wsp<long long>(a, lay.off_hsum);
  s.bpre = wsp<long long>(a, lay.off_bpre);
  s.boff = wsp<uint32_t>(a, lay.off_boff);
  s.tot = wsp<long long>(a, lay.off_tot);
  s.keys = wsp<unsigned long long>(a, lay.off_keys);
  s.keys2 = wsp<unsigned long long>(a, lay.off_keys2);
  s.fail_count = wsp<uint32_t>(a, lay.off_fail);
  s.fail_list = wsp<uint32_t>(a, lay.off_fail) + 64;
  s.desc = wsp<int4>(a, lay.off_desc);
  s.t = wsp<float>(a, pl.kernel == KSUM_LAPLACIAN ? lay.off_t2 : lay.off_t1);
  s.perm = a.perm_out ? a.perm_out + (int64_t)a.p0 * lay.L : nullptr;
  s.cneg = pl.sort_const;
  s.deriv = a.deriv ? 1 : 0;
  s.nch = lay.sort_nch;
  s.chunk = lay.sort_chunk;
  const unsigned g1 = (unsigned)xcd_grid((int64_t)a.nsl * lay.sort_nch);
  if (!a.reuse_front) {   // histogram, scan and scatter do not depend on the derivative mode
    mark(a, ST_SORT_HIST);
    sort_hist_kernel<<<g1, 512, 0, a.stream>>>(s);
    mark(a, ST_SORT_SCAN);
    sort_scan_kernel<<<a.nsl, 1024, 0, a.stream>>>(s);
    mark(a, ST_SORT_SCATTER);
    const int64_t chunk = lay.sort_chunk;
    if ((chunk + 12287) / 12288 < (chunk + 8191) / 8192)
      sort_scatter_kernel<12288><<<g1, kScatThreads, 0, a.stream>>>(s);
    else
      sort_scatter_kernel<8192><<<g1, kScatThreads, 0, a.stream>>>(s);
  } else {
    // the scan, which clears the fallback list, does not run: clear it here
    mark(a, ST_MISC);
    const hipError_t e = launch_fill_zero(reinterpret_cast<float *>(s.fail_count), 1, a.stream);
    if (e != hipSuccess) return e;
  }
  const int64_t items = (int64_t)a.nsl * lay.sort_groups;
  const unsigned g4 = (unsigned)std::min<int64_t>(xcd_grid(items), 256 * 2);
  mark(a, ST_SORT_GROUP);
  if (a.deriv)
    sort_fast_kernel<true><<<g4, kFThreads, 0, a.stream>>>(s);
  else
    sort_fast_kernel<false><<<g4, kFThreads, 0, a.stream>>>(s);
  mark(a, ST_SORT_FALLBACK);
  sort_fallback_kernel<<<256, 256, 0, a.stream>>>(s);
  return hipGetLastError();
}

}  // namespace ksum
