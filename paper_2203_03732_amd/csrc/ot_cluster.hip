// Optimal transport with the copies of every point kept as clusters
// (Section 4, Lemma 4.1).
//
// The reduction is that of ot.hip (theta = 4 max(n_b, n_a) / eps, supplies
// rounded down and demands up into unit copies), but no copy is stored. By
// Lemma 4.1 the copies of a point hold at most two duals, one step apart,
// so a supply point b is described by Y_b (the larger dual, where its F_b
// free copies sit after the free-copy raise) and a demand point a by Z_a
// (its larger dual; G_a of its copies are free, at 0). A matched pair of
// copies is tight (eq. (2)), so its supply copy's dual is fixed by its
// demand copy's; the pairs between b and a are counted in two slots, by the
// parity of the demand copy's level (Z_a and Z_a - 1 differ in parity, so a
// level change of a point never moves a count between slots).
//
// A phase, point by point:
//   (I)   the free copies of b all sit at Y_b, so edge (a, b) is admissible
//         exactly when k + 1 = Z_a + Y_b (the lower level of a never is,
//         by (I1) on its upper level). The admissible points of each b with
//         free copies are listed once per phase, in b's scan order. Then
//         synchronous rounds: every b still looking proposes to the first
//         listed point with top-level copies left, asking for all its
//         looking copies; a point serves its proposers in ascending b, each
//         as far as its top copies go; a b served in part or not at all
//         goes on after that point, one that runs out of points stops.
//   (II)  a point hands out the top copies taken in the phase: its free
//         copies first, then those matched at Z_a in ascending order of
//         their partner's point, whose partner copies become free.
//   (III) the taken copies drop to Z_a - 1 (if all top copies went, Z_a
//         itself drops); a b with copies left over rises one step (Y_b + 1),
//         and its evicted copies take the largest dual of their point.
// The phases stop once at most T supply copies are free. Then the free
// supply copies take free demand copies in point order (north-west corner on
// the counts), and the plan kernels of ot.hip turn the pair counts into the
// plan.
//
// Workgroup 0 of the loop holds the points' state: the demand points' levels
// and capacities and the supply points' duals in LDS, each supply point's
// round state in the registers of the thread that owns it, the pair counts
// and a bitmap of each demand point's partners in global memory. With every
// step of a round separated by a workgroup barrier, a round costs a few
// hundred nanoseconds instead of a grid-wide barrier. Listing the admissible
// points reads every row with free copies (n_a rounded costs each), which
// one workgroup cannot do fast enough: it publishes the rows and the demand
// levels, and every workgroup of the grid lists a share of the rows into a
// global staging area, which workgroup 0 then copies into its LDS when it
// fits. The two hand-overs per phase are a flag and an arrival counter,
// each wait bounded.
#include "internal.h"
#include "device_common.h"

namespace prot {
namespace {

constexpr int kCT = 1024;                                // threads per workgroup
constexpr int kPerMax = (int)(kClusterMaxPoints / kCT);  // supply points per thread
constexpr int32_t kNever = 0x40000000;                   // a level no edge reaches
constexpr uint32_t kDone = 0xFFFFFFFFu;                  // epoch: the loop has ended
// Bounded waits of the hand-overs: ~2 s of the 100 MHz device clock (a phase
// takes microseconds); on time-out bit 5 of the error word is raised and
// every workgroup leaves.
constexpr int64_t kWaitTicks = 200000000ll;

// Hand-over words (each on its own 256-byte line of ClusterArgs::sync; the
// entries staged in phase p are counted in word kSyncStaged + p % 2).
// 64-bit: (phase published by workgroup 0, kDone at the end) << 32 | its rows
constexpr int kEpoch = 0;
// 64-bit: (workgroups done listing) << 40 | (list entries they staged), both
// cumulative over the phases
constexpr int kArrive = 64;
constexpr unsigned long long kStagedMask = (1ull << 40) - 1ull;

// LDS of workgroup 0 (32-bit words), for n_a demand and n_b supply points;
// the demand arrays have n_a rounded up to 8 entries. req holds, while the
// lists are built, each demand point's top level (kNever if it has no top
// copies), read 8 at a time; the other workgroups keep only that array.
struct Lds {
    int32_t *Z, *top, *bot, *cap, *req, *minb, *G;  // n_a each
    int32_t *Y, *evict;                         // n_b each
    uint16_t *list;                             // the rest: the phase's lists
    int64_t list_cap;
};

__device__ inline Lds lds_layout(char *base, int64_t n_b, int64_t n_a, int64_t bytes)
{
    Lds L;
    const int64_t na8 = (n_a + 7) & ~7ll;
    int32_t *p = reinterpret_cast<int32_t *>(base);
    L.Z = p;
    L.top = p + na8;
    L.bot = p + 2 * na8;
    L.cap = p + 3 * na8;
    L.req = p + 4 * na8;
    L.minb = p + 5 * na8;
    L.G = p + 6 * na8;
    L.Y = p + 7 * na8;
    L.evict = L.Y + n_b;
    const int64_t used = ((7 * na8 + 2 * n_b) * 4 + 15) & ~15ll;
    L.list = reinterpret_cast<uint16_t *>(base + used);
    L.list_cap = (bytes - used) / 2;
    return L;
}

// Column of scan position j of supply point b.
__device__ inline int col_of(int b, int j, int n_a, int origin)
{
    if (origin != 0) return j;
    const int a = b % n_a + j;
    return a >= n_a ? a - n_a : a;
}

// Block-wide sum (all threads call); the result is valid in every thread.
__device__ long long block_sum64(long long v, long long *red)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int wv = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[wv] = v;
    __syncthreads();
    long long t = 0;
    for (int i = 0; i < kCT / 64; ++i) t += red[i];
    return t;
}

// Whether pred holds in any thread of the workgroup, with one barrier
// (all threads call, the same number of times). Call c raises flag c % 4 and
// reads it after the barrier; thread 0 clears flag (c + 2) % 4 before it:
// its readers (call c - 2) passed the barrier of call c - 1 before, its
// writers (call c + 2) come after the barrier of call c + 1.
__device__ inline int block_any(int pred, int *flags, uint32_t &calls)
{
    const uint32_t c = calls++;
    if (threadIdx.x == 0) flags[(c + 2) & 3] = 0;
    if (__ballot(pred) && (threadIdx.x & 63) == 0) flags[c & 3] = 1;
    __syncthreads();
    return flags[c & 3];
}

// Thread 0 waits until *word >= want (or holds kDone, for the epoch), or
// for the arrival word until its count field reaches want; false on
// time-out (err bit 5 raised).
template <class W>
__device__ bool wait_at_least(W *word, W want, Ctl *ctl, W *seen, int shift = 0)
{
    const int64_t t0 = (int64_t)wall_clock64();
    for (int spins = 0;; ++spins) {
        const W v = ld_agent(word);
        if ((v >> shift) >= want) {
            *seen = v;
            return true;
        }
        if ((spins & 63) == 63 && (int64_t)wall_clock64() - t0 > kWaitTicks) {
            __hip_atomic_fetch_or(&ctl->err, 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *seen = shift ? ((W)kDone << shift) : (W)kDone;
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Every store that another workgroup reads is an agent-scope store (coherent
// across the chip's caches without a cache write-back); a wave waits for its
// stores to complete before the workgroup barrier that precedes a flag.
__device__ inline void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Bit e set iff k[e] - zt[e] == need (k: 8 int16 in kv, zt: 8 levels).
__device__ inline uint32_t level_hits(uint4 kv, int4 z0, int4 z1, int need)
{
    const uint32_t kw[4] = {kv.x, kv.y, kv.z, kv.w};
    const int z[8] = {z0.x, z0.y, z0.z, z0.w, z1.x, z1.y, z1.z, z1.w};
    uint32_t m = 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int kk = (int)(int16_t)((kw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
        m |= (uint32_t)(kk - z[e] == need) << e;
    }
    return m;
}

constexpr int kSegVisits = 128;  // chunk visits per row per step (2 per lane)

// The admissible lists of rows [0, count) of this workgroup's share (row i:
// supply point rb[i], whose free copies sit at rneed[i] + 1), each in its scan
// order: column a is admissible when k - Z_a = need and a has top copies
// (zt holds Z_a, or kNever). A wave takes kRowsPerWave rows at once; in a
// step, lane l looks at chunks (8 columns) 2l and 2l + 1 of each row's
// visit order, which starts at the chunk holding the row's first column,
// wraps around, and ends with that chunk again (its columns below the
// start), so lane order is scan order. A row's entries (scan positions) go
// to a block of the staging area taken with one atomic; its offset and
// length to loff[b], llen[b]. Rows longer than one step (n_a > 1016) are
// read twice: once to count, once to write.
template <int kRowsPerWave, class RowAt>
__device__ void build_lists(const ClusterArgs &A, const int32_t *zt, int count, RowAt row_at,
                            int *total, int32_t *staged)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n_a = A.n_a, nch = (n_a + 7) >> 3, V = nch + 1;
    const int nseg = (V + kSegVisits - 1) / kSegVisits;
    for (int r0 = wave * kRowsPerWave; r0 < count; r0 += (kCT / 64) * kRowsPerWave) {
        int b[kRowsPerWave], s0[kRowsPerWave], c0[kRowsPerWave], need[kRowsPerWave];
        int len[kRowsPerWave], off[kRowsPerWave];
#pragma unroll
        for (int g = 0; g < kRowsPerWave; ++g) {
            b[g] = -1;
            need[g] = 0;
            if (r0 + g < count) row_at(r0 + g, &b[g], &need[g]);
            s0[g] = (b[g] >= 0 && A.origin == 0) ? b[g] % n_a : 0;
            c0[g] = s0[g] >> 3;
            len[g] = 0;
            off[g] = 0;
        }
        // pass 0 counts (rows of several steps), pass 1 writes; a one-step
        // row is counted and written from the same registers
        for (int pass = nseg == 1 ? 1 : 0; pass < 2; ++pass) {
            int run[kRowsPerWave];
#pragma unroll
            for (int g = 0; g < kRowsPerWave; ++g) run[g] = 0;
            for (int seg = 0; seg < nseg; ++seg) {
                uint4 kv[kRowsPerWave][2];
                int cc[kRowsPerWave][2];
#pragma unroll
                for (int g = 0; g < kRowsPerWave; ++g)
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int v = seg * kSegVisits + lane * 2 + u;
                        int c = c0[g] + v;
                        if (c >= nch) c -= nch;
                        cc[g][u] = c;
                        kv[g][u] = make_uint4(0, 0, 0, 0);
                        if (b[g] >= 0 && v < V)
                            kv[g][u] = *reinterpret_cast<const uint4 *>(
                                A.k + (int64_t)b[g] * A.ldk + c * 8);
                    }
                uint32_t m[kRowsPerWave][2];
#pragma unroll
                for (int g = 0; g < kRowsPerWave; ++g)
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int v = seg * kSegVisits + lane * 2 + u;
                        m[g][u] = 0;
                        if (b[g] < 0 || v >= V) continue;
                        const int c = cc[g][u];
                        const int4 z0 = *reinterpret_cast<const int4 *>(zt + c * 8);
                        const int4 z1 = *reinterpret_cast<const int4 *>(zt + c * 8 + 4);
                        const int lo = v == 0 ? s0[g] : 0;
                        const int hi = v == nch ? s0[g] : n_a;
                        m[g][u] =
                            level_hits(kv[g][u], z0, z1, need[g]) & range_mask(c * 8, lo, hi);
                    }
#pragma unroll
                for (int g = 0; g < kRowsPerWave; ++g) {
                    if (b[g] < 0) continue;  // the whole wave
                    const int mine = __builtin_popcount(m[g][0]) + __builtin_popcount(m[g][1]);
                    int incl = mine;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int t = __shfl_up(incl, o);
                        if (lane >= o) incl += t;
                    }
                    const int seg_len = __shfl(incl, 63);
                    if (pass == 0) {
                        len[g] += seg_len;
                        continue;
                    }
                    if (nseg == 1) {
                        len[g] = seg_len;
                        int x = 0;
                        if (lane == 0 && seg_len > 0) x = add_agent(staged, seg_len);
                        off[g] = __shfl(x, 0);
                    }
                    int at = off[g] + run[g] + incl - mine;
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        uint32_t mm = m[g][u];
                        while (mm) {
                            const int e = __builtin_ctz(mm);
                            mm &= mm - 1u;
                            int j = cc[g][u] * 8 + e - s0[g];  // (a - s0) mod n_a
                            if (j < 0) j += n_a;
                            st_agent(A.stage + at++, (uint16_t)j);
                        }
                    }
                    run[g] += seg_len;
                }
            }
            if (pass == 0) {
#pragma unroll
                for (int g = 0; g < kRowsPerWave; ++g) {
                    int x = 0;
                    if (lane == 0 && b[g] >= 0 && len[g] > 0) x = add_agent(staged, len[g]);
                    off[g] = __shfl(x, 0);
                }
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int g = 0; g < kRowsPerWave; ++g)
                if (b[g] >= 0) {
                    st_agent(A.loff + b[g], off[g]);
                    st_agent(A.llen + b[g], len[g]);
                    atomicAdd(total, len[g]);
                }
        }
    }
}

// Workgroups other than 0: wait for a phase, list a share of its rows,
// arrive; until workgroup 0 ends the loop.
// Workgroups other than 0 list the rows (workgroup 0 only when it is alone).
// A share of the rows, and the demand levels, are read into LDS together.
template <int kRows>
__device__ void helper_loop(const ClusterArgs &A, char *lds_raw)
{
    __shared__ uint32_t s_epoch;
    __shared__ int s_rows, s_total;
    const int na8 = (A.n_a + 7) & ~7;
    int32_t *zt = reinterpret_cast<int32_t *>(lds_raw);
    int32_t *rb = zt + na8, *rneed = rb + A.n_b;
    const int H = gridDim.x - 1, w = blockIdx.x - 1;
    for (uint32_t ph = 1;; ++ph) {
        if (threadIdx.x == 0) {
            unsigned long long e;
            wait_at_least<unsigned long long>(reinterpret_cast<unsigned long long *>(A.sync + kEpoch),
                                              ph, A.ctl, &e, 32);
            s_epoch = (uint32_t)(e >> 32);
            s_rows = (int)(uint32_t)e;
            s_total = 0;
        }
        __syncthreads();
        if (s_epoch == kDone) return;
        const int n = s_rows;
        const int lo = (int)((int64_t)n * w / H), cnt = (int)((int64_t)n * (w + 1) / H) - lo;
        for (int a = threadIdx.x; a < na8; a += kCT) zt[a] = ld_agent(A.zt + a);
        for (int i = threadIdx.x; i < cnt; i += kCT) {
            rb[i] = ld_agent(A.act + lo + i);
            rneed[i] = ld_agent(A.need + lo + i);
        }
        __syncthreads();
        build_lists<kRows>(A, zt, cnt, [&](int i, int *b, int *need) {
            *b = rb[i];
            *need = rneed[i];
        }, &s_total, A.staged + (ph & 1));
        stores_done();
        __syncthreads();
        if (threadIdx.x == 0)
            add_agent(reinterpret_cast<unsigned long long *>(A.sync + kArrive),
                      (1ull << 40) | (unsigned long long)s_total);
    }
}

// kPer supply points per thread (b = tid + s * kCT), kRows rows listed at
// once by a wave: (2, 2) up to 2048 supply points, (4, 1) up to 4096 (more
// registers per thread leave room for fewer rows in flight).
template <int kPer, int kRows>
__global__ void __launch_bounds__(kCT) cluster_loop_kernel(ClusterArgs A)
{
    extern __shared__ __align__(16) char lds_raw[];
    if (blockIdx.x != 0) {
        helper_loop<kRows>(A, lds_raw);
        return;
    }
    __shared__ long long red[kCT / 64];
    __shared__ int n_act, lds_lists, s_abort, s_total, s_staged;
    __shared__ unsigned long long ph_scanned, ph_matched;
    __shared__ int any_flags[4];
    uint32_t any_calls = 0;
    Lds L = lds_layout(lds_raw, A.n_b, A.n_a, A.lds_bytes);
    const int tid = threadIdx.x;
    const int n_b = A.n_b, n_a = A.n_a;
    const uint32_t P = gridDim.x;

    // the state: cold start (every copy free, y(b) = 1, y(a) = 0)
    const int na8 = (n_a + 7) & ~7;
    for (int a = tid; a < na8; a += kCT) {
        const int32_t d = a < n_a ? (int32_t)(A.d_off[a + 1] - A.d_off[a]) : 0;
        L.Z[a] = 0;
        L.top[a] = d;
        L.bot[a] = 0;
        L.minb[a] = 0x7FFFFFFF;
        L.G[a] = d;
    }
    for (int b = tid; b < n_b; b += kCT) {
        L.Y[b] = 1;
        L.evict[b] = 0;
    }
    if (tid == 0) s_abort = 0;
    if (tid < 4) any_flags[tid] = 0;
    int32_t F[kPer], want[kPer], pos[kPer], li[kPer], tgt[kPer], jp[kPer], loff[kPer],
        llen[kPer];
    bool act[kPer], prop[kPer], contest[kPer];
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
        const int b = tid + s * kCT;
        F[s] = b < n_b ? (int32_t)(A.s_off[b + 1] - A.s_off[b]) : 0;
    }
    long long phases = 0, sum_free = 0, rounds = 0, max_rounds = 0, scanned = 0;
    int status = 0;
    long long n_free = 0;
    unsigned long long staged_before = 0;  // entries staged in earlier phases (thread 0)
    for (;;) {
        long long mine = 0;
#pragma unroll
        for (int s = 0; s < kPer; ++s) mine += F[s];
        n_free = block_sum64(mine, red);
        if (n_free <= A.T) break;
        if (A.max_phases > 0 && phases == A.max_phases) {
            status = 1;
            break;
        }
        if (A.phase_bound > 0 && phases >= A.phase_bound) {
            status = 2;
            break;
        }
        phases += 1;
        sum_free += n_free;

        // Step (I): publish the rows with free copies and the demand levels
        if (tid == 0) {
            n_act = 0;
            s_total = 0;
            ph_scanned = 0;
            ph_matched = 0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            if (b < n_b && F[s] > 0) {
                const int r = atomicAdd(&n_act, 1);
                st_agent(A.act + r, b);
                st_agent(A.need + r, L.Y[b] - 1);
            }
        }
        for (int a = tid; a < na8; a += kCT) {
            const int32_t z = L.top[a] > 0 ? L.Z[a] : kNever;
            L.req[a] = z;
            st_agent(A.zt + a, z);
        }
        // (the staging count of the next phase starts at zero: it was last
        // used in the previous phase, which every workgroup has finished)
        if (tid == 0) st_agent(A.staged + ((phases + 1) & 1), 0);
        stores_done();
        __syncthreads();
        if (tid == 0)
            st_agent(reinterpret_cast<unsigned long long *>(A.sync + kEpoch),
                     ((unsigned long long)phases << 32) | (uint32_t)n_act);
        // ... the other workgroups list the rows (this one only when alone) ...
        if (P == 1) {
            build_lists<kRows>(A, L.req, n_act, [&](int i, int *b, int *need) {
                *b = ld_agent(A.act + i);
                *need = ld_agent(A.need + i);
            }, &s_total, A.staged + (phases & 1));
            stores_done();
            __syncthreads();
        }
        if (tid == 0) {
            int staged = s_total;
            if (P > 1) {
                unsigned long long seen;
                if (!wait_at_least<unsigned long long>(
                        reinterpret_cast<unsigned long long *>(A.sync + kArrive),
                        (unsigned long long)(P - 1) * (unsigned long long)phases, A.ctl, &seen, 40))
                    s_abort = 1;
                staged = (int)((seen & kStagedMask) - staged_before);
                staged_before = seen & kStagedMask;
            }
            s_staged = staged;
            lds_lists = (int64_t)((staged + 7) & ~7) <= L.list_cap;
        }
        // (each supply point's list block, read while thread 0 waits)
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            act[s] = b < n_b && F[s] > 0;
        }
        __syncthreads();
        if (s_abort) {
            status = 3;
            break;
        }
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            loff[s] = act[s] ? ld_agent(A.loff + b) : 0;
            llen[s] = act[s] ? ld_agent(A.llen + b) : 0;
        }
        // ... and take the staged lists into LDS when they fit
        if (lds_lists) {
            const int staged = s_staged;
            const uint32_t *src = reinterpret_cast<const uint32_t *>(A.stage);
            uint32_t *dst = reinterpret_cast<uint32_t *>(L.list);
            for (int i = tid; i < (staged + 1) / 2; i += kCT) dst[i] = ld_agent(src + i);
        }
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            want[s] = F[s];
            pos[s] = 0;
            li[s] = 0;
        }
        for (int a = tid; a < na8; a += kCT) {
            L.cap[a] = L.top[a];
            L.req[a] = 0;
        }
        __syncthreads();
        const bool in_lds = lds_lists;

        long long ph_rounds = 0;
        for (;;) {
            // (i) propose, against the capacities at the round's start
            long long my_scan = 0;
            int my_prop = 0;
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                prop[s] = false;
                if (!act[s]) continue;
                const int b = tid + s * kCT;
                int i = li[s], a = -1, j = -1;
                for (; i < llen[s]; ++i) {
                    j = in_lds ? L.list[loff[s] + i] : ld_agent(A.stage + loff[s] + i);
                    a = col_of(b, j, n_a, A.origin);
                    if (L.cap[a] > 0) break;
                }
                li[s] = i;
                if (i >= llen[s]) {
                    my_scan += n_a - pos[s];
                    act[s] = false;
                    continue;
                }
                my_scan += j - pos[s] + 1;
                pos[s] = j;
                jp[s] = j;
                tgt[s] = a;
                prop[s] = true;
                my_prop = 1;
                atomicAdd(&L.req[a], want[s]);
            }
            if (my_scan) atomicAdd(&ph_scanned, (unsigned long long)my_scan);
            if (!block_any(my_prop, any_flags, any_calls)) break;
            ph_rounds += 1;
            // (ii) a point asked for no more than it has serves everyone;
            // the others serve in ascending b
            // (the lowest contending b of each such point is selected at once)
            int my_contest = 0;
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                contest[s] = prop[s] && L.req[tgt[s]] > L.cap[tgt[s]];
                if (contest[s]) atomicMin(&L.minb[tgt[s]], tid + s * kCT);
                my_contest |= contest[s];
            }
            const int contested = block_any(my_contest, any_flags, any_calls);
            int32_t grant[kPer];
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                grant[s] = 0;
                if (prop[s] && !contest[s]) {
                    grant[s] = want[s];
                    atomicSub(&L.cap[tgt[s]], want[s]);
                }
            }
            if (contested) {
                for (;;) {
                    // the selected b is served as far as the point's copies go
#pragma unroll
                    for (int s = 0; s < kPer; ++s) {
                        if (!contest[s] || L.minb[tgt[s]] != tid + s * kCT) continue;
                        const int a = tgt[s];
                        const int32_t g = want[s] < L.cap[a] ? want[s] : L.cap[a];
                        L.cap[a] -= g;
                        grant[s] = g;
                        contest[s] = false;
                        L.minb[a] = 0x7FFFFFFF;
                    }
                    __syncthreads();
                    // the rest of a point with nothing left get nothing; the
                    // others select their next lowest b
                    int left = 0;
#pragma unroll
                    for (int s = 0; s < kPer; ++s) {
                        if (!contest[s]) continue;
                        if (L.cap[tgt[s]] == 0) {
                            contest[s] = false;
                        } else {
                            atomicMin(&L.minb[tgt[s]], tid + s * kCT);
                            left = 1;
                        }
                    }
                    if (!block_any(left, any_flags, any_calls)) break;
                }
            }
            // (iii) the grants become pairs (at the demand copies' next level)
            long long my_match = 0;
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                if (!prop[s]) continue;
                const int b = tid + s * kCT;
                const int a = tgt[s];
                L.req[a] = 0;
                const int32_t g = grant[s];
                if (g > 0) {
                    int2 *cell = A.w + (int64_t)b * n_a + a;
                    atomicAdd(((L.Z[a] - 1) & 1) == 0 ? &cell->x : &cell->y, g);
                    atomicOr(A.mask + (int64_t)a * A.nwb + (b >> 6), 1ull << (b & 63));
                    atomicOr(A.msum + a, 1ull << (b >> 6));
                    my_match += g;
                }
                want[s] -= g;
                if (want[s] == 0) {
                    act[s] = false;
                } else {
                    pos[s] = jp[s] + 1;
                    li[s] += 1;
                }
            }
            if (my_match) atomicAdd(&ph_matched, (unsigned long long)my_match);
            __syncthreads();
        }

        // Step (II): each point hands out the top copies taken
        for (int a = tid; a < n_a; a += kCT) {
            const int32_t taken = L.top[a] - L.cap[a];
            if (taken == 0) continue;
            const int32_t z = L.Z[a];
            int32_t rem = taken;
            if (z == 0) {
                const int32_t g = L.G[a];
                const int32_t u = rem < g ? rem : g;
                L.G[a] = g - u;
                rem -= u;
            }
            const int p = z & 1;
            unsigned long long *mrow = A.mask + (int64_t)a * A.nwb;
            const unsigned long long sum0 = rem > 0 ? A.msum[a] : 0ull;
            unsigned long long words = sum0, sum = sum0;
            // partners in ascending b: four bitmap words, then four pair
            // cells, loaded at once
            while (words && rem > 0) {
                int wd[4];
                unsigned long long wv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    wd[q] = -1;
                    wv[q] = 0ull;
                    if (words) {
                        wd[q] = __builtin_ctzll(words);
                        words &= words - 1ull;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (wd[q] >= 0) wv[q] = mrow[wd[q]];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (wd[q] < 0 || rem == 0) continue;
                    unsigned long long bits = wv[q], keep = bits;
                    while (bits && rem > 0) {
                        int bb[4];
                        int2 cv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            bb[u] = -1;
                            if (bits) {
                                bb[u] = wd[q] * 64 + __builtin_ctzll(bits);
                                bits &= bits - 1ull;
                            }
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            cv[u] = bb[u] >= 0 ? A.w[(int64_t)bb[u] * n_a + a] : make_int2(0, 0);
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (bb[u] < 0 || rem == 0) continue;
                            int32_t &c = p ? cv[u].y : cv[u].x;
                            if (c == 0) continue;
                            const int32_t e = rem < c ? rem : c;
                            c -= e;
                            rem -= e;
                            A.w[(int64_t)bb[u] * n_a + a] = cv[u];
                            atomicAdd(&L.evict[bb[u]], e);
                            if (cv[u].x == 0 && cv[u].y == 0) keep &= ~(1ull << (bb[u] & 63));
                        }
                    }
                    if (keep != wv[q]) {
                        mrow[wd[q]] = keep;
                        if (!keep) sum &= ~(1ull << wd[q]);
                    }
                }
            }
            if (sum != sum0) A.msum[a] = sum;
            // step (III a)
            if (L.cap[a] == 0) {
                L.Z[a] = z - 1;
                L.top[a] = L.bot[a] + taken;
                L.bot[a] = 0;
            } else {
                L.top[a] = L.cap[a];
                L.bot[a] += taken;
            }
        }
        __syncthreads();
        // Step (III b) and the raise
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            if (b >= n_b) continue;
            if (want[s] > 0) L.Y[b] += 1;
            F[s] = want[s] + L.evict[b];
            L.evict[b] = 0;
        }
        rounds += ph_rounds;
        max_rounds = ph_rounds > max_rounds ? ph_rounds : max_rounds;
        scanned += (long long)ph_scanned;
        if (A.trace && phases <= kTraceCap && tid == 0) {
            long long *t = A.trace + 4 * (phases - 1);
            t[0] = n_free;
            t[1] = ph_rounds;
            t[2] = (long long)ph_scanned;
            t[3] = (long long)ph_matched;
        }
        __syncthreads();
    }
    // the other workgroups leave
    if (tid == 0)
        st_agent(reinterpret_cast<unsigned long long *>(A.sync + kEpoch),
                 (unsigned long long)kDone << 32);

    // the state the later kernels read
    for (int a = tid; a < n_a; a += kCT) {
        A.G[a] = L.G[a];
        A.Zo[a] = L.Z[a];
        A.topo[a] = L.top[a];
        A.boto[a] = L.bot[a];
    }
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
        const int b = tid + s * kCT;
        if (b < n_b) {
            A.Yo[b] = L.Y[b];
            A.Fo[b] = F[s];
        }
    }
    if (tid == 0) {
        Ctl *c = A.ctl;
        c->phases = phases;
        c->sum_free = sum_free;
        c->rounds = rounds;
        c->max_rounds = max_rounds;
        c->scanned = (unsigned long long)scanned;
        c->status = status == 3 ? 1 : status;  // an aborted loop is not complete
        c->free_after = n_free;
    }
}

// Pair counts per (b, a) = both slots, and the partial sums of k over them.
constexpr int kCntThreads = 256;
__global__ void __launch_bounds__(kCntThreads) cluster_count_kernel(ClusterArgs A, int32_t *cnt,
                                                                    long long *part_k)
{
    __shared__ long long sk[kCntThreads];
    long long mine = 0;
    const int64_t total = (int64_t)A.n_b * A.n_a;
    for (int64_t e = blockIdx.x * (int64_t)kCntThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kCntThreads) {
        const int2 v = A.w[e];
        const int32_t c = v.x + v.y;
        cnt[e] = c;
        if (c) {
            const int64_t b = e / A.n_a, a = e - b * A.n_a;
            mine += (long long)c * A.k[b * A.ldk + a];
        }
    }
    sk[threadIdx.x] = mine;
    __syncthreads();
    for (int off = kCntThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sk[threadIdx.x] += sk[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part_k[blockIdx.x] = sk[0];
}

// The completion: free supply copies (in point order) take free demand
// copies (in point order), north-west corner on the counts F and G. One
// workgroup; adds the pairs to cnt and their k to part_k[0].
__global__ void __launch_bounds__(kCT) cluster_complete_kernel(ClusterArgs A, int32_t *cnt,
                                                               long long *part_k, int run)
{
    __shared__ long long red[kCT / 64];
    __shared__ long long tmp[kCT];
    if (!run || A.ctl->status != 0) return;
    // running totals of F over b and of G over a, each thread a contiguous slice
    const int tid = threadIdx.x;
    auto scan = [&](const int32_t *v, int n, int64_t *out) {
        const int per = (n + kCT - 1) / kCT;
        const int lo = tid * per, hi = lo + per < n ? lo + per : n;
        long long s = 0;
        for (int i = lo; i < hi; ++i) s += v[i];
        tmp[tid] = s;
        __syncthreads();
        for (int off = 1; off < kCT; off <<= 1) {
            const long long add = tid >= off ? tmp[tid - off] : 0;
            __syncthreads();
            tmp[tid] += add;
            __syncthreads();
        }
        long long run_ = tmp[tid] - s;
        for (int i = lo; i < hi; ++i) {
            out[i] = run_;
            run_ += v[i];
        }
        if (tid == kCT - 1) out[n] = tmp[kCT - 1];
        __syncthreads();
    };
    scan(A.Fo, A.n_b, A.PF);
    scan(A.G, A.n_a, A.PG);
    __threadfence_block();
    __syncthreads();
    long long mine = 0;
    for (int b = tid; b < A.n_b; b += kCT) {
        long long f0 = A.PF[b], f1 = A.PF[b + 1];
        if (f1 == f0) continue;
        // first a whose range [PG[a], PG[a+1]) ends after f0
        int lo = 0, hi = A.n_a - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (A.PG[mid + 1] > f0) hi = mid;
            else lo = mid + 1;
        }
        for (int a = lo; a < A.n_a && A.PG[a] < f1; ++a) {
            const long long x0 = f0 > A.PG[a] ? f0 : A.PG[a];
            const long long x1 = f1 < A.PG[a + 1] ? f1 : A.PG[a + 1];
            if (x1 <= x0) continue;
            cnt[(int64_t)b * A.n_a + a] += (int32_t)(x1 - x0);
            mine += (x1 - x0) * (long long)A.k[(int64_t)b * A.ldk + a];
        }
    }
    const long long t = block_sum64(mine, red);
    if (tid == 0) part_k[0] += t;
}

// Duals in the two-cluster form: for each point the smaller dual of its
// copies and how many copies hold it (the others hold one more); points
// without copies give 0 and 0. Supply point b: its copies below Y_b are
// those of pairs whose demand copy's level puts them at Y_b - 1 (one wave
// per point, reading its row of pair counts). A supply copy outside
// {Y_b - 1, Y_b} would break Lemma 4.1: err bit 7.
__global__ void __launch_bounds__(256) cluster_duals_b_kernel(ClusterArgs A, int32_t *lo_out,
                                                              int32_t *nlo_out)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= A.n_b) return;
    const int lane = threadIdx.x & 63;
    const int32_t Y = A.Yo[b];
    long long lo = 0;
    bool bad = false;
    for (int a = lane; a < A.n_a; a += 64) {
        const int2 v = A.w[(int64_t)b * A.n_a + a];
        if (v.x == 0 && v.y == 0) continue;
        const int32_t z = A.Zo[a];
        const int32_t kk = A.k[(int64_t)b * A.ldk + a];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int32_t c = p ? v.y : v.x;
            if (!c) continue;
            const int32_t lev = (z & 1) == p ? z : z - 1;
            const int32_t yb = kk - lev;
            if (yb == Y - 1) lo += c;
            else if (yb != Y) bad = true;
        }
    }
    for (int off = 32; off > 0; off >>= 1) lo += __shfl_xor(lo, off);
    if (__ballot(bad) && lane == 0)
        __hip_atomic_fetch_or(&A.ctl->err, 128, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (lane == 0) {
        const long long s = A.s_off[b + 1] - A.s_off[b];
        if (s == 0) {
            lo_out[b] = 0;
            nlo_out[b] = 0;
        } else if (lo > 0) {
            lo_out[b] = Y - 1;
            nlo_out[b] = (int32_t)lo;
        } else {
            lo_out[b] = Y;
            nlo_out[b] = (int32_t)s;
        }
    }
}

__global__ void cluster_duals_a_kernel(ClusterArgs A, int32_t *lo_out, int32_t *nlo_out)
{
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < A.n_a; a += gridDim.x * blockDim.x) {
        const long long d = A.d_off[a + 1] - A.d_off[a];
        const int32_t z = A.Zo[a], top = A.topo[a], bot = A.boto[a];
        if ((long long)top + bot != d)
            __hip_atomic_fetch_or(&A.ctl->err, 128, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (d == 0) {
            lo_out[a] = 0;
            nlo_out[a] = 0;
        } else if (bot > 0) {
            lo_out[a] = z - 1;
            nlo_out[a] = bot;
        } else {
            lo_out[a] = z;
            nlo_out[a] = (int32_t)d;
        }
    }
}

__global__ void cluster_zero_kernel(unsigned long long *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

}  // namespace

int64_t cluster_lds_fixed(int64_t n_b, int64_t n_a)
{
    const int64_t na8 = (n_a + 7) & ~7ll;
    return ((7 * na8 + 2 * n_b) * 4 + 15) & ~15ll;
}

hipError_t launch_cluster_init(const ClusterArgs &A, hipStream_t s)
{
    // pair counts and partner bitmaps start at zero
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(1024), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(A.w), (int64_t)A.n_b * A.n_a);
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(256), dim3(256), 0, s, A.mask,
                       (int64_t)A.n_a * A.nwb);
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(16), dim3(256), 0, s, A.msum, (int64_t)A.n_a);
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(1), dim3(128), 0, s,
                       reinterpret_cast<unsigned long long *>(A.sync), (int64_t)kSyncWords / 2);
    static bool attr_set = false;
    if (!attr_set) {
        for (const void *fn : {(const void *)cluster_loop_kernel<2, 2>,
                               (const void *)cluster_loop_kernel<kPerMax, 1>}) {
            const hipError_t e = hipFuncSetAttribute(
                fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kClusterLdsBytes);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    return hipGetLastError();
}

const void *cluster_loop_fn(int32_t n_b)
{
    return n_b <= 2 * kCT ? (const void *)cluster_loop_kernel<2, 2>
                          : (const void *)cluster_loop_kernel<kPerMax, 1>;
}

hipError_t cluster_grid(int32_t n_b, int *grid)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cluster_loop_fn(n_b), kCT,
                                                                (size_t)kClusterLdsBytes);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    // about one batch of rows (16 waves x 2 rows) per workgroup when every
    // supply point has free copies
    int want = (n_b + 31) / 32;
    const int most = per_cu * cus;
    *grid = want < 1 ? 1 : (want > most ? most : want);
    return hipSuccess;
}

hipError_t launch_cluster_loop(const ClusterArgs &A, int grid, hipStream_t s)
{
    ClusterArgs copy = A;
    void *args[] = {&copy};
    return hipLaunchCooperativeKernel(cluster_loop_fn(A.n_b), dim3(grid), dim3(kCT), args,
                                      (unsigned)A.lds_bytes, s);
}

hipError_t launch_cluster_counts(const ClusterArgs &A, int32_t *cnt, long long *part_k, int complete,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(cluster_count_kernel, dim3(kFinalizeBlocks), dim3(kCntThreads), 0, s, A,
                       cnt, part_k);
    hipLaunchKernelGGL(cluster_complete_kernel, dim3(1), dim3(kCT), 0, s, A, cnt, part_k,
                       complete);
    return hipGetLastError();
}

hipError_t launch_cluster_duals(const ClusterArgs &A, int32_t *b_lo, int32_t *b_nlo, int32_t *a_lo,
                                int32_t *a_nlo, hipStream_t s)
{
    hipLaunchKernelGGL(cluster_duals_b_kernel, dim3((unsigned)((A.n_b + 3) / 4)), dim3(256), 0, s, A,
                       b_lo, b_nlo);
    hipLaunchKernelGGL(cluster_duals_a_kernel, dim3((unsigned)((A.n_a + 255) / 256)), dim3(256), 0,
                       s, A, a_lo, a_nlo);
    return hipGetLastError();
}

}  // namespace prot
