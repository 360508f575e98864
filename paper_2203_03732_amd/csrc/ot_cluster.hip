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
// Everything the phases touch lives in one workgroup: the demand points'
// levels and capacities and the supply points' duals in LDS, each supply
// point's round state in the registers of the thread that owns it, the
// admissible lists in LDS while they fit (else in a global overflow area),
// the pair counts and a bitmap of each demand point's partners in global
// memory (read back through this workgroup's cache). With the state of a
// point held by one thread and every step of a round separated by a
// workgroup barrier, a round costs a few hundred nanoseconds instead of a
// grid-wide barrier, which is what the O(n^2 / eps^2) method needs at the
// few thousand points it is meant for.
#include "internal.h"
#include "device_common.h"

namespace prot {
namespace {

constexpr int kCT = 1024;                            // threads of the cluster loop
constexpr int kPer = (int)(kClusterMaxPoints / kCT);  // points per thread
constexpr int kVisits = 2;                           // 8-column chunks per lane per step
constexpr uint32_t kGlobalList = 0x80000000u;        // list info: the row's list is global

// LDS layout (32-bit words), for n_a demand and n_b supply points.
struct Lds {
    int32_t *Z, *top, *bot, *cap, *req, *minb;  // n_a each
    int32_t *Y, *evict;                         // n_b each
    uint32_t *linfo;                            // n_b: list base and length
    uint16_t *act;                              // n_b: supply points with free copies
    uint16_t *list;                             // the rest: admissible scan positions
    int64_t list_cap;
};

__device__ inline Lds lds_layout(char *base, int64_t n_b, int64_t n_a, int64_t bytes)
{
    Lds L;
    int32_t *p = reinterpret_cast<int32_t *>(base);
    L.Z = p;
    L.top = p + n_a;
    L.bot = p + 2 * n_a;
    L.cap = p + 3 * n_a;
    L.req = p + 4 * n_a;
    L.minb = p + 5 * n_a;
    L.Y = p + 6 * n_a;
    L.evict = L.Y + n_b;
    L.linfo = reinterpret_cast<uint32_t *>(L.evict + n_b);
    L.act = reinterpret_cast<uint16_t *>(L.linfo + n_b);
    const int64_t used = (6 * n_a + 3 * n_b) * 4 + ((n_b * 2 + 15) & ~15ll);
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

__device__ inline int list_at(const ClusterArgs &A, const Lds &L, int b, uint32_t info, int i)
{
    if (info & kGlobalList) return A.list[(int64_t)b * A.n_a + i];
    return L.list[(info >> 13) + i];
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

// The admissible list of supply point b (free copies at y) in its scan
// order, built by one wave: lane l looks at chunks (8 columns) l * kVisits
// .. of the visit order, which starts at the chunk holding b's first
// column, wraps around, and ends with that chunk again (its columns below
// the start).
__device__ void build_list(const ClusterArgs &A, Lds &L, int b, int y, int *lds_used)
{
    const int lane = threadIdx.x & 63;
    const int n_a = A.n_a;
    const int s0 = A.origin == 0 ? b % n_a : 0;
    const int nch = (n_a + 7) >> 3, c0 = s0 >> 3;
    const int V = nch + 1;
    const int need = y - 1;  // k + 1 == Z + y  <=>  k - Z == y - 1
    const int16_t *krow = A.k + (int64_t)b * A.ldk;
    constexpr int kMaxSteps = (int)((kClusterMaxPoints / 8 + 1 + 64 * kVisits - 1) / (64 * kVisits));
    uint32_t bits[kMaxSteps][kVisits];
    int excl[kMaxSteps];  // entries before this lane's chunks within each step
    int step_base[kMaxSteps];
    const int steps = (V + 64 * kVisits - 1) / (64 * kVisits);
    int len = 0;
#pragma unroll
    for (int st = 0; st < kMaxSteps; ++st) {
        excl[st] = 0;
        step_base[st] = len;
        if (st >= steps) continue;
        int mine = 0;
#pragma unroll
        for (int u = 0; u < kVisits; ++u) {
            const int v = (st * 64 + lane) * kVisits + u;
            uint32_t m = 0;
            if (v < V) {
                int c = c0 + v;
                if (c >= nch) c -= nch;
                const int col0 = c * 8;
                const uint4 kv = *reinterpret_cast<const uint4 *>(krow + col0);
                const uint32_t kw[4] = {kv.x, kv.y, kv.z, kv.w};
                const int lo = v == 0 ? s0 : 0;
                const int hi = v == nch ? s0 : n_a;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int a = col0 + e;
                    if (a < lo || a >= hi) continue;
                    const int kk = (int)(int16_t)((kw[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
                    if (L.top[a] > 0 && kk - L.Z[a] == need) m |= 1u << e;
                }
            }
            bits[st][u] = m;
            mine += __builtin_popcount(m);
        }
        // prefix of the lanes' counts within the step (lane order = visit order)
        int incl = mine;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        excl[st] = incl - mine;
        len += __shfl(incl, 63);
    }
    int base = 0;
    uint32_t info = kGlobalList;
    if (lane == 0 && len > 0) {
        const int at = atomicAdd(lds_used, len);
        if ((int64_t)at + len <= L.list_cap) info = ((uint32_t)at << 13);
    }
    info = __shfl(info, 0);
    if (!(info & kGlobalList)) base = (int)(info >> 13);
    if (lane == 0) L.linfo[b] = len == 0 ? 0u : (info | (uint32_t)len);
    // the scan position of column a is (a - s0) mod n_a
#pragma unroll
    for (int st = 0; st < kMaxSteps; ++st) {
        if (st >= steps) break;
        int at = step_base[st] + excl[st];
#pragma unroll
        for (int u = 0; u < kVisits; ++u) {
            uint32_t m = bits[st][u];
            if (!m) continue;
            const int v = (st * 64 + lane) * kVisits + u;
            int c = c0 + v;
            if (c >= nch) c -= nch;
            while (m) {
                const int e = __builtin_ctz(m);
                m &= m - 1u;
                int j = c * 8 + e - s0;
                if (j < 0) j += n_a;
                if (info & kGlobalList) A.list[(int64_t)b * n_a + at] = (uint16_t)j;
                else L.list[base + at] = (uint16_t)j;
                ++at;
            }
        }
    }
}

__global__ void __launch_bounds__(kCT) cluster_loop_kernel(ClusterArgs A)
{
    extern __shared__ __align__(16) char lds_raw[];
    __shared__ long long red[kCT / 64];
    __shared__ int n_act, lds_used;
    __shared__ unsigned long long ph_scanned, ph_matched;
    Lds L = lds_layout(lds_raw, A.n_b, A.n_a, A.lds_bytes);
    const int tid = threadIdx.x;
    const int n_b = A.n_b, n_a = A.n_a;

    // the state: cold start (every copy free, y(b) = 1, y(a) = 0)
    for (int a = tid; a < n_a; a += kCT) {
        const int32_t d = (int32_t)(A.d_off[a + 1] - A.d_off[a]);
        L.Z[a] = 0;
        L.top[a] = d;
        L.bot[a] = 0;
        L.minb[a] = 0x7FFFFFFF;
        L.req[a] = 0;
        A.G[a] = d;
    }
    for (int b = tid; b < n_b; b += kCT) {
        L.Y[b] = 1;
        L.evict[b] = 0;
    }
    int32_t F[kPer], want[kPer], pos[kPer], li[kPer], tgt[kPer], jp[kPer];
    uint32_t info[kPer];
    bool act[kPer], prop[kPer], contest[kPer];
#pragma unroll
    for (int s = 0; s < kPer; ++s) {
        const int b = tid + s * kCT;
        F[s] = b < n_b ? (int32_t)(A.s_off[b + 1] - A.s_off[b]) : 0;
    }
    long long phases = 0, sum_free = 0, rounds = 0, max_rounds = 0, scanned = 0;
    int status = 0;
    long long n_free = 0;
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

        // Step (I): the admissible lists of the points with free copies
        if (tid == 0) {
            n_act = 0;
            lds_used = 0;
            ph_scanned = 0;
            ph_matched = 0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            if (b < n_b && F[s] > 0) L.act[atomicAdd(&n_act, 1)] = (uint16_t)b;
        }
        __syncthreads();
        for (int r = tid >> 6; r < n_act; r += kCT / 64) {
            const int b = L.act[r];
            build_list(A, L, b, L.Y[b], &lds_used);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPer; ++s) {
            const int b = tid + s * kCT;
            want[s] = F[s];
            pos[s] = 0;
            li[s] = 0;
            act[s] = b < n_b && F[s] > 0;
            info[s] = act[s] ? L.linfo[b] : 0u;
        }
        for (int a = tid; a < n_a; a += kCT) L.cap[a] = L.top[a];
        __syncthreads();

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
                const int len = (int)(info[s] & 0x1FFFu);
                int i = li[s], a = -1, j = -1;
                for (; i < len; ++i) {
                    j = list_at(A, L, b, info[s], i);
                    a = col_of(b, j, n_a, A.origin);
                    if (L.cap[a] > 0) break;
                }
                li[s] = i;
                if (i >= len) {
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
            if (!__syncthreads_or(my_prop)) break;
            ph_rounds += 1;
            // (ii) a point asked for no more than it has serves everyone;
            // the others serve in ascending b
            int my_contest = 0;
#pragma unroll
            for (int s = 0; s < kPer; ++s) {
                contest[s] = prop[s] && L.req[tgt[s]] > L.cap[tgt[s]];
                my_contest |= contest[s];
            }
            const int contested = __syncthreads_or(my_contest);
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
#pragma unroll
                    for (int s = 0; s < kPer; ++s)
                        if (contest[s]) atomicMin(&L.minb[tgt[s]], tid + s * kCT);
                    __syncthreads();
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
                    int left = 0;
#pragma unroll
                    for (int s = 0; s < kPer; ++s) {
                        if (contest[s] && L.cap[tgt[s]] == 0) contest[s] = false;  // nothing left
                        left |= contest[s];
                    }
                    if (!__syncthreads_or(left)) break;
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
                    if (((L.Z[a] - 1) & 1) == 0) cell->x += g;
                    else cell->y += g;
                    atomicOr(A.mask + (int64_t)a * A.nwb + (b >> 6), 1ull << (b & 63));
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
                const int32_t g = A.G[a];
                const int32_t u = rem < g ? rem : g;
                A.G[a] = g - u;
                rem -= u;
            }
            const int p = z & 1;
            unsigned long long *mrow = A.mask + (int64_t)a * A.nwb;
            for (int wd = 0; wd < A.nwb && rem > 0; ++wd) {
                unsigned long long bits = mrow[wd], keep = bits;
                while (bits && rem > 0) {
                    const int b = wd * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1ull;
                    int2 *cell = A.w + (int64_t)b * n_a + a;
                    int2 v = *cell;
                    int32_t &c = p ? v.y : v.x;
                    if (c == 0) continue;
                    const int32_t e = rem < c ? rem : c;
                    c -= e;
                    rem -= e;
                    *cell = v;
                    atomicAdd(&L.evict[b], e);
                    if (v.x == 0 && v.y == 0) keep &= ~(1ull << (b & 63));
                }
                if (keep != mrow[wd]) mrow[wd] = keep;
            }
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

    // the state the later kernels read
    for (int a = tid; a < n_a; a += kCT) {
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
        c->status = status;
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
    return (6 * n_a + 3 * n_b) * 4 + ((n_b * 2 + 15) & ~15ll);
}

hipError_t launch_cluster_init(const ClusterArgs &A, hipStream_t s)
{
    // pair counts and partner bitmaps start at zero
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(1024), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long *>(A.w), (int64_t)A.n_b * A.n_a);
    hipLaunchKernelGGL(cluster_zero_kernel, dim3(256), dim3(256), 0, s, A.mask,
                       (int64_t)A.n_a * A.nwb);
    static bool attr_set = false;
    if (!attr_set) {
        const hipError_t e = hipFuncSetAttribute((const void *)cluster_loop_kernel,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)kClusterLdsBytes);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    return hipGetLastError();
}

hipError_t launch_cluster_loop(const ClusterArgs &A, hipStream_t s)
{
    hipLaunchKernelGGL(cluster_loop_kernel, dim3(1), dim3(kCT), (size_t)A.lds_bytes, s, A);
    return hipGetLastError();
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
