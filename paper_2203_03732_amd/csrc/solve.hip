// The integer phase loop of arXiv:2203.03732, Section 2.2, on one GPU.
//
// One persistent launch runs every phase (a plain launch; a gate at its
// start admits the resident workgroups, see the kernel). Per phase:
//   B'  (the free supply rows) is the list F[p & 1];
//   step (I), a maximal matching M' in the admissible graph of B', is built
//       by synchronous proposal rounds: every row still looking scans its row
//       of the rounded-cost matrix (starting at its own column and wrapping,
//       or at column 0) for the first column that is admissible,
//       k[b][a] + 1 == y(a) + y(b), and was not taken before the round began;
//       it proposes with an atomic max on that column's 64-bit key (the
//       round above, the row below in reverse order, so the lowest-index
//       proposer of the round wins; the row's dual rides in the low bits);
//   step (II) and (III) need no separate pass: the key of a column always
//       names its current mate, so the first proposal to a column in a
//       round appends the old mate (if any) to the next free list and the
//       column to the list of columns taken this phase, and a row that finds
//       nothing raises its own dual and re-enters the next free list.
// One grid barrier ends each round. A round in which no workgroup saw a lost
// proposal (or no proposal was made) ends the phase: M' is maximal.
//
// y(a) is stored as t(a) = -y(a) >= 0, the number of phases in which column a
// was taken. Each workgroup keeps t in LDS. The columns taken in a round are
// read back by every workgroup at the start of the next round and marked
// there (bit 15 of t, which makes k + t exceed any y(b) - 1), so the scan
// itself needs no global memory besides the matrix row; their t is raised by
// one at the same time (Section 2.2 lowers y(a) after the greedy step, and a
// marked column is not looked at again in the phase), and the marks are
// cleared when the phase ends.
//
// Communication between workgroups uses device-scope atomics and loads and
// write-through stores only, so a round needs no L2 write-back or invalidate:
//   * each round has one 64-bit word that every workgroup adds to once; the
//     sum packs the arrivals, the workgroups that lost a proposal and the
//     numbers of taken columns and freed rows, and the value returned to a
//     workgroup is the prefix of the workgroups that arrived before it, which
//     places its list entries;
//   * list entries are written after the arrival, tagged with the phase, and
//     a reader waits (bounded) until the entry carries the expected tag;
//   * a row re-enters the free list with its dual packed beside it, so a
//     phase start needs no load of y(b); y(b) is also stored (for the
//     results), and the wave waits for that store to complete before it
//     writes the row's next free-list entry;
//   * when the last round of a phase is over, the poll that saw it also
//     lays out the next free list, so a phase boundary costs one workgroup
//     barrier besides the rounds'.
#include "device_common.h"
#include "internal.h"

namespace prot {
namespace {

constexpr int kWave = 64;
constexpr int kChunk = kWave * 8;   // columns examined per wave per load
constexpr int kPrefetch = 6;        // chunks in flight in a long scan
constexpr int kSlotBatch = 4;       // rows whose first chunks are loaded together
constexpr int kTeamPrefetch = 4;    // chunks in flight per wave of a team scan

// Round words: workgroup w adds to word w % G of the round; each word sums
// over the workgroups of its group that arrived.
constexpr int kShiftFree = 21, kShiftLose = 42, kShiftArrive = 53;
constexpr unsigned long long kField = (1ull << 21) - 1;
constexpr uint16_t kTaken = 0x8000;            // mark: column taken earlier in the phase
constexpr int kSpinLimit = 1 << 22;            // bounded waits for list entries
// Bounded wait at a round barrier: ~10 s of the 100 MHz device clock. A round
// of the largest instances takes milliseconds; on time-out bit 5 of the error
// word is raised and every workgroup leaves the loop (each one's wait is
// bounded, so the grid drains).
constexpr int64_t kBarrierTicks = 1000000000ll;
constexpr int32_t kDualMax = 0x7FFF;           // t (-y(a)) fits its 15-bit field
constexpr int kGateSpin = 256;                 // gate polls (~0.3 ms) before it closes early

// Waits until this wave's earlier stores and atomics have completed.
__device__ inline void wait_memory()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Value of a tagged list entry ((tag << 32) | value) once it carries `tag`.
// The wait is bounded: on time-out bit 2 of the error word is raised and the
// value is used as found. take_raw_from starts from a value v already loaded
// from p and returns the 32-bit payload as found; take_entry_from and
// take_entry clamp it to a row or column in [0, n).
__device__ inline uint32_t take_raw_from(const unsigned long long *p, unsigned long long v,
                                        uint32_t tag, int32_t *err)
{
    for (int spins = 0; (uint32_t)(v >> 32) != tag; v = ld_agent(p)) {
        // once any wait has timed out, later waits give up at once
        if (++spins > kSpinLimit || ((spins & 1023) == 0 && (ld_agent(err) & 36))) {
            __hip_atomic_fetch_or(err, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return (uint32_t)v;
}

// y(b) + 1 for a row that found no column (step (III)), unless that leaves
// the field the dual travels in (dual_max, see RowPack): then bit 6 of the
// error word is raised, the dual stays and -1 is returned: the row is left
// out of the next free list, so the loop ends soon and the host reports the
// error (Lemma 3.2 keeps |y| <= K + 2 in every state the method reaches, and
// the host admits only K + 2 <= dual_max, so only an inconsistent warm start
// gets here).
__device__ inline int32_t grown_dual(int32_t yb, int32_t dual_max, int32_t *err)
{
    if (yb < dual_max) return yb + 1;
    __hip_atomic_fetch_or(err, 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return -1;
}

// t(a) + 1 for a column taken in a phase (step (III)), with the same guard.
__device__ inline uint16_t grown_t(uint16_t t, int32_t *err)
{
    if ((t & 0x7FFF) < kDualMax) return (uint16_t)(t + 1);
    __hip_atomic_fetch_or(err, 64, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return t;
}

__device__ inline int32_t take_entry_from(const unsigned long long *p, unsigned long long v,
                                         uint32_t tag, int n, int32_t *err)
{
    const int32_t x = (int32_t)take_raw_from(p, v, tag, err);
    return x < 0 ? 0 : (x >= n ? n - 1 : x);
}

__device__ inline int32_t take_entry(const unsigned long long *p, uint32_t tag, int n, int32_t *err)
{
    return take_entry_from(p, ld_agent(p), tag, n, err);
}

// Group j holding position i of a list split into group regions, given the
// exclusive prefix sums pre[0..G) of the region lengths.
__device__ inline int group_of(const uint32_t *pre, int G, uint32_t i)
{
    int j = 0;
    while (j + 1 < G && pre[j + 1] <= i) ++j;
    return j;
}

__device__ inline uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline int wave_min(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}

__device__ inline uint32_t wave_exclusive_scan(uint32_t v, int lane)
{
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x - v;
}

// The largest dual among a point's copies (the transport reduction), tagged
// with the phase that set it: a device-scope atomic max, complete before the
// workgroup's arrival like the y(b) store it follows.
__device__ inline void raise_top(unsigned long long *p, int64_t phase, int32_t v)
{
    const unsigned long long w = ((unsigned long long)(phase + 1) << 32) | (uint32_t)v;
    __hip_atomic_fetch_max(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The largest dual of a point's copies after the previous phase, read in
// phase `phase` (a copy that found nothing in this phase already moved the
// word to this phase's value, one more).
__device__ inline int32_t top_before(unsigned long long w, int64_t phase)
{
    const int32_t m = (int32_t)(uint32_t)w;
    return (int64_t)(w >> 32) == phase + 1 ? m - 1 : m;
}

__device__ inline unsigned long long tagged(uint32_t tag, int32_t v)
{
    return ((unsigned long long)tag << 32) | (uint32_t)v;
}

// A row and its dual travel together (|y| <= K + 2, Lemma 3.2): a column's
// key is (round << (15 + rb)) | (mask - b) << 15 | y(b), so the larger key
// wins a round and within a round the smaller b; the free lists hold
// y(b) << rb | b. A row that enters a phase, or is evicted, thus brings its
// dual with it and nobody loads y(b). rb = 17 row bits (up to 131,071 rows;
// duals up to 32,767; round ids below 2^32) or 18 (up to 262,143 rows;
// duals up to 16,383; round ids below 2^31).
struct RowPack {
    uint32_t rb, mask;
    int32_t dual_max;
    uint32_t round_limit;
};
__device__ inline RowPack row_pack(int32_t wide)
{
    return wide ? RowPack{18u, (1u << 18) - 1u, 0x3FFF, 0x7FFFFF00u}
                : RowPack{17u, (1u << 17) - 1u, 0x7FFF, 0xFFFFFF00u};
}
constexpr uint32_t kNoRow = 0xFFFFFFFFu;

__device__ inline unsigned long long make_key(uint32_t r, int32_t b, int32_t y, const RowPack &P)
{
    return ((unsigned long long)r << (15 + P.rb)) |
           ((unsigned long long)(P.mask - (uint32_t)b) << 15) | ((uint32_t)y & 0x7FFFu);
}
__device__ inline int32_t key_row(unsigned long long k, const RowPack &P)
{
    return (int32_t)(P.mask - ((uint32_t)(k >> 15) & P.mask));
}
__device__ inline uint32_t key_free(unsigned long long k, const RowPack &P)
{
    return (((uint32_t)k & 0x7FFFu) << P.rb) | (uint32_t)key_row(k, P);
}
__device__ inline uint32_t free_val(int32_t b, int32_t y, const RowPack &P)
{
    return ((uint32_t)y << P.rb) | (uint32_t)b;
}

// First admissible, unmarked column of this chunk (wave-wide, lowest column
// first); -1 if none.
__device__ inline int chunk_hit(int col0, uint4 kv, uint4 tv, int need, int lo, int hi)
{
    const uint32_t cand = col0 < hi ? (match_mask(kv, tv, need) & range_mask(col0, lo, hi)) : 0u;
    const unsigned long long cb = __ballot(cand != 0u);
    if (cb == 0ull) return -1;
    const int L = __builtin_ctzll(cb);
    return __builtin_amdgcn_readlane(col0, L) + __builtin_ctz(__builtin_amdgcn_readlane(cand, L));
}

// Scan position j of row b visits column (origin + j) mod n, so a scan from
// position pos covers the column ranges [origin + pos, n) and then
// [0, origin), or only [origin + pos - n, origin).
// (Two named ranges rather than an array, so that selecting one with a
// runtime index stays in registers.)
struct Segs {
    int lo0, hi0, lo1, hi1;
    __device__ int lo(int sg) const { return sg ? lo1 : lo0; }
    __device__ int hi(int sg) const { return sg ? hi1 : hi0; }
};

__device__ inline Segs segments(int n, int origin, int pos)
{
    Segs s;
    const int c0 = origin + pos;
    if (c0 < n) {
        s.lo0 = c0; s.hi0 = n; s.lo1 = 0; s.hi1 = origin;
    } else {
        s.lo0 = c0 - n; s.hi0 = origin; s.lo1 = 0; s.hi1 = 0;
    }
    return s;
}

// Where the scan of slot s (held by lane s of the wave) starts this round.
struct SlotView {
    int b, pos, yb, origin;
    int rb;         // the row of costs b reads (b, or the point a copy copies)
    Segs S;
    int sg, base;   // first nonempty segment (1 if none) and its first chunk
};

__device__ inline SlotView slot_view(int s, int s_b, int s_pos, int s_yb, int origin_mode, int n,
                                     int s_rb)
{
    SlotView v;
    v.b = __builtin_amdgcn_readlane(s_b, s);
    v.rb = __builtin_amdgcn_readlane(s_rb, s);
    v.pos = __builtin_amdgcn_readlane(s_pos, s);
    v.yb = __builtin_amdgcn_readlane(s_yb, s);
    v.origin = origin_mode == 0 ? v.b : 0;
    v.S = segments(n, v.origin, v.pos);
    v.sg = v.S.lo0 < v.S.hi0 ? 0 : 1;
    v.base = v.S.lo(v.sg) & ~7;
    return v;
}

__device__ inline Hit hit_at(int a, int origin, int n)
{
    return Hit{a >= origin ? a - origin : a - origin + n, a};
}

// Where the loop's rounded costs come from. MatrixSrc reads the int16 matrix;
// PointsSrc<D> (point sets of dimension D) computes the same integers from
// the points with the cost build's operations (sqdist, fast_k, refine_k with
// the instance's threshold table), so no n x n matrix is stored or read.
// chunk(row, col0) gives k for columns col0 .. col0 + 7 (col0 a multiple of
// 8, col0 < n), 0x7FFF past n.
struct MatrixSrc {
    static constexpr int kAhead = kPrefetch;      // chunks in flight in a long scan
    static constexpr int kTeamAhead = kTeamPrefetch;
    static constexpr int kBatch = kSlotBatch;     // rows whose first chunks go together
    const int16_t *k;
    int64_t ldk;
    using Row = const int16_t *;
    __device__ Row row(int b) const { return k + (int64_t)b * ldk; }
    __device__ uint4 chunk(const Row &r, int col0) const
    {
        return *reinterpret_cast<const uint4 *>(r + col0);
    }
};

// The same matrix stored as bytes (every cost at most K <= 253; padding 0xFF,
// which exceeds every y(b) - 1 and so is never admissible): half the bytes
// per entry. A chunk is 8 bytes, widened to the int16 layout of MatrixSrc.
struct MatrixSrc8 {
    static constexpr int kAhead = kPrefetch;
    static constexpr int kTeamAhead = kTeamPrefetch;
    static constexpr int kBatch = kSlotBatch;
    const uint8_t *k;
    int64_t ldk;
    using Row = const uint8_t *;
    __device__ Row row(int b) const { return k + (int64_t)b * ldk; }
    __device__ uint4 chunk(const Row &r, int col0) const
    {
        const uint2 v = *reinterpret_cast<const uint2 *>(r + col0);
        // bytes c0 c1 c2 c3 -> halfwords c0, c1 and c2, c3 (byte 0x0C of the
        // selector gives zero)
        return uint4{__builtin_amdgcn_perm(0u, v.x, 0x0c010c00u),
                     __builtin_amdgcn_perm(0u, v.x, 0x0c030c02u),
                     __builtin_amdgcn_perm(0u, v.y, 0x0c010c00u),
                     __builtin_amdgcn_perm(0u, v.y, 0x0c030c02u)};
    }
};

template <int D>
struct PointsSrc {
    // computing ahead buys less than loading ahead and costs 8 * D registers
    // per chunk
    static constexpr int kAhead = 2;
    static constexpr int kTeamAhead = 2;
    static constexpr int kBatch = 2;
    const float *X, *Y, *th;
    float inv, delta;
    int K, n;
    struct Row {
        float x[D];
    };
    __device__ Row row(int b) const
    {
        Row r;
#pragma unroll
        for (int q = 0; q < D; ++q) r.x[q] = X[(int64_t)b * D + q];
        return r;
    }
    __device__ uint4 chunk(const Row &r, int col0) const
    {
        float y[8 * D];
        if (col0 + 8 <= n) {
            // 8 points = 2D float4 (col0 is a multiple of 8, so aligned)
            const float4 *p = reinterpret_cast<const float4 *>(Y + (int64_t)col0 * D);
#pragma unroll
            for (int i = 0; i < 2 * D; ++i) {
                const float4 v = p[i];
                y[4 * i] = v.x;
                y[4 * i + 1] = v.y;
                y[4 * i + 2] = v.z;
                y[4 * i + 3] = v.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8 * D; ++i) y[i] = col0 + i / D < n ? Y[(int64_t)col0 * D + i] : 0.0f;
        }
        int g[8];
        float sv[8];
        bool all_ok = true;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            bool ok;
            sv[e] = sqdist<D>(r.x, y + e * D, D);
            g[e] = fast_k(sv[e], inv, delta, K, ok);
            all_ok &= ok;
        }
        if (!all_ok) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                bool ok;
                fast_k(sv[e], inv, delta, K, ok);
                if (!ok) g[e] = refine_k(sv[e], g[e], K, th);
            }
        }
        if (col0 + 8 > n) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (col0 + e >= n) g[e] = 0x7FFF;
        }
        uint4 w;
        w.x = (uint32_t)(uint16_t)g[0] | ((uint32_t)(uint16_t)g[1] << 16);
        w.y = (uint32_t)(uint16_t)g[2] | ((uint32_t)(uint16_t)g[3] << 16);
        w.z = (uint32_t)(uint16_t)g[4] | ((uint32_t)(uint16_t)g[5] << 16);
        w.w = (uint32_t)(uint16_t)g[6] | ((uint32_t)(uint16_t)g[7] << 16);
        return w;
    }
};

template <int D>
__device__ inline PointsSrc<D> points_src(const LoopArgs &A)
{
    // the same m, K, 1/(m eps) and margin as the cost build's pass 2
    PointsSrc<D> s;
    const float mf = *A.pm;
    s.X = A.px;
    s.Y = A.py;
    s.th = A.pth;
    s.K = (mf > 0.0f) ? (int32_t)floor(1.0 / A.peps) : 0;
    s.inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * A.peps)) : 0.0f;
    s.delta = classify_margin(s.K);
    s.n = A.n_a;
    return s;
}

// Continue the wave-cooperative scan of a row in segment sg at column base
// (a multiple of 8), kPrefetch chunks in flight; the duals come from LDS.
template <int AHEAD, class Src>
__device__ Hit scan_from(const Src &src, const typename Src::Row &row, const uint16_t *t_lds,
                         int n, int origin, const Segs &S, int sg, int base, int need, int lane,
                         int *mn)
{
    for (; sg < 2; ++sg) {
        const int slo = S.lo(sg), shi = S.hi(sg);
        if (slo >= shi) {
            base = -1;
            continue;
        }
        if (base < 0) base = slo & ~7;
        while (base < shi) {
            uint4 kv[AHEAD];
#pragma unroll
            for (int u = 0; u < AHEAD; ++u) {
                const int col0 = base + u * kChunk + lane * 8;
                kv[u] = make_uint4(0u, 0u, 0u, 0u);
                if (col0 < shi) kv[u] = src.chunk(row, col0);
            }
#pragma unroll
            for (int u = 0; u < AHEAD; ++u) {
                const int col0 = base + u * kChunk + lane * 8;
                uint4 tv = make_uint4(0u, 0u, 0u, 0u);
                if (col0 < shi) tv = *reinterpret_cast<const uint4 *>(t_lds + col0);
                if (mn && col0 < shi)
                    *mn = min(*mn, min_sum_masked(kv[u], tv, range_mask(col0, slo, shi)));
                const int a = chunk_hit(col0, kv[u], tv, need, slo, shi);
                if (a >= 0) return hit_at(a, origin, n);
            }
            base += AHEAD * kChunk;
        }
        base = -1;
    }
    return Hit{-1, -1};
}

// Team scan: R waves of one workgroup share a row. The row's chunks (kChunk
// columns, segment 0 first, then segment 1, each aligned down to 8 columns)
// are dealt out round-robin, chunk c to wave c mod R; wave k = this wave's
// rank. Returns the scan position of this wave's first hit (its chunks are
// visited in order), or kNoHit. The first pass loads one chunk per wave;
// later passes kTeamPrefetch each, and stop once the team's best hit so far
// (*best, in LDS) precedes them.
constexpr int kNoHit = 0x7FFFFFFF;

template <class Src>
__device__ int team_scan(const Src &src, const typename Src::Row &row, const uint16_t *t_lds,
                         int n, int origin, const Segs &S, int need, int k, int R, int lane,
                         const int *best, int *mn)
{
    const int b0 = S.lo0 & ~7, b1 = S.lo1 & ~7;
    const int nc0 = S.lo0 < S.hi0 ? (S.hi0 - b0 + kChunk - 1) / kChunk : 0;
    const int nc1 = S.lo1 < S.hi1 ? (S.hi1 - b1 + kChunk - 1) / kChunk : 0;
    const int nc = nc0 + nc1;
    int c = k;
    int depth = 1;
    while (c < nc) {
        uint4 kv[Src::kTeamAhead];
#pragma unroll
        for (int u = 0; u < Src::kTeamAhead; ++u) {
            const int cc = c + u * R;
            kv[u] = make_uint4(0u, 0u, 0u, 0u);
            if (u < depth && cc < nc) {
                const bool s1 = cc >= nc0;
                const int col0 = (s1 ? b1 + (cc - nc0) * kChunk : b0 + cc * kChunk) + lane * 8;
                if (col0 < (s1 ? S.hi1 : S.hi0)) kv[u] = src.chunk(row, col0);
            }
        }
#pragma unroll
        for (int u = 0; u < Src::kTeamAhead; ++u) {
            const int cc = c + u * R;
            if (u >= depth || cc >= nc) break;
            const bool s1 = cc >= nc0;
            const int lo = s1 ? S.lo1 : S.lo0, hi = s1 ? S.hi1 : S.hi0;
            const int col0 = (s1 ? b1 + (cc - nc0) * kChunk : b0 + cc * kChunk) + lane * 8;
            uint4 tv = make_uint4(0u, 0u, 0u, 0u);
            if (col0 < hi) tv = *reinterpret_cast<const uint4 *>(t_lds + col0);
            if (mn && col0 < hi) *mn = min(*mn, min_sum_masked(kv[u], tv, range_mask(col0, lo, hi)));
            const int a = chunk_hit(col0, kv[u], tv, need, lo, hi);
            if (a >= 0) return hit_at(a, origin, n).j;
        }
        c += depth * R;
        depth = Src::kTeamAhead;
        if (c < nc) {
            // first scan position of chunk c
            const bool s1 = c >= nc0;
            const int col = s1 ? max(S.lo1, b1 + (c - nc0) * kChunk) : max(S.lo0, b0 + c * kChunk);
            const int j = hit_at(col, origin, n).j;
            if (__hip_atomic_load(best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < j) break;
        }
    }
    return kNoHit;
}

__global__ void loop_reset_kernel(LoopArgs a)
{
    Ctl *c = a.ctl;
    for (int i = 0; i < 3 * kMaxGroups; ++i) a.words[i * kWordStride] = 0ull;
    c->gate_count = 0;
    c->gate = 0;
    c->free0 = 0;
    c->scanned = 0;
    c->status = 0;
    c->phases = c->sum_free = c->rounds = c->max_rounds = 0;
    c->free_after = 0;
    if (a.trace)
        for (int i = 0; i < 4; ++i) a.trace[i] = 0;
}


// Initial state: y(b) = 1, y(a) = 0, M empty (Section 2.2), or a warm start.
// The free list of the first phase goes to F[0] with the launch's first tag
// (one past the last tag of the previous launch), its length to ctl->free0.
// A cold start also does the work of loop_reset_kernel (in block 0) and sets
// every mate_b to -1 for the decode after the loop.
__global__ void init_kernel(LoopArgs a, int32_t warm, const int32_t *mate_a,
                            int32_t *mate_b, const int32_t *y_a)
{
    if (!warm && blockIdx.x == 0 && threadIdx.x < 3 * kMaxGroups)
        a.words[threadIdx.x * kWordStride] = 0ull;
    if (!warm && blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl *c = a.ctl;
        c->gate_count = 0;
        c->gate = 0;
        c->scanned = 0;
        c->status = 0;
        c->phases = c->sum_free = c->rounds = c->max_rounds = 0;
        c->free_after = 0;
        if (a.trace)
            for (int i = 0; i < 4; ++i) a.trace[i] = 0;
    }
    const int n = a.n, na = a.n_a;  // rows, columns
    const int lane = threadIdx.x & 63;
    const uint32_t tag0 = a.ctl->tag_last + 1u;
    const RowPack P = row_pack(a.wide);
    const int top = a.n_pad > n ? a.n_pad : n;
    for (int base = blockIdx.x * blockDim.x; base < top; base += gridDim.x * blockDim.x) {
        const int i = base + threadIdx.x;
        bool is_free = false;
        if (i < na) {
            if (!warm) {
                a.key[i] = 0ull;
                a.t[i] = 0;
            } else {
                const int32_t m = mate_a[i];
                a.key[i] = m >= 0 ? make_key(0u, m, a.y_b[m], P) : 0ull;
                a.t[i] = (uint16_t)(-y_a[i]);
            }
        } else if (i < a.n_pad) {
            a.t[i] = 0;
        }
        if (i < n) {
            if (a.skip) a.skip[i] = 0u;
            if (!warm) {
                a.y_b[i] = 1;
                a.F[0][i] = tagged(tag0, (int32_t)free_val(i, 1, P));
                mate_b[i] = -1;
            } else {
                is_free = mate_b[i] < 0;
            }
        }
        if (warm) {
            const unsigned long long bal = __ballot(is_free);
            if (bal) {
                uint32_t at = 0;
                if (lane == 0) at = add_agent(&a.ctl->free0, (uint32_t)__popcll(bal));
                at = __builtin_amdgcn_readfirstlane(at);
                if (is_free)
                    a.F[0][at + lanes_below(bal)] =
                        tagged(tag0, (int32_t)free_val(i, a.y_b[i], P));
            }
        }
    }
    if (!warm && blockIdx.x == 0 && threadIdx.x == 0) a.ctl->free0 = (uint32_t)n;
}

// Warm-start check, O(n): the mate arrays form one matching, (I1) holds
// (y(b) >= 0, y(a) <= 0, y(a) = 0 for a free a; Section 2.2) and every dual
// lies within Lemma 3.2's bound |y| <= K + 2 = ybound.
__global__ void check_state_kernel(int64_t n, int64_t na, const int32_t *mate_a,
                                   const int32_t *mate_b, const int32_t *y_a,
                                   const int32_t *y_b, int32_t ybound, Ctl *ctl)
{
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < na;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t ma = mate_a[i];
        if (ma >= n || ma < -1) bad = true;
        else if (ma >= 0 && mate_b[ma] != i) bad = true;
        if (y_a[i] > 0 || y_a[i] < -ybound) bad = true;
        if (ma < 0 && y_a[i] != 0) bad = true;
        if (i < n) {
            const int32_t mb = mate_b[i];
            if (mb >= na || mb < -1) bad = true;
            else if (mb >= 0 && mate_a[mb] != i) bad = true;
            if (y_b[i] < 0 || y_b[i] > ybound) bad = true;
        }
    }
    if (bad) __hip_atomic_fetch_or(&ctl->err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Warm-start check, O(n_b n_a): (I2), i.e. eq. (2) on every edge and eq. (3)
// on the matching, in units of eps: y(a) + y(b) <= k + 1 for every (a, b) and
// y(a) + y(b) = k for a matched pair (Section 2.2). One thread per 8 columns
// of a row; rows by grid.y.
__global__ void check_feasible_kernel(const int16_t *k, int64_t ldk, int64_t n, int64_t na,
                                      const int32_t *mate_b, const int32_t *y_a,
                                      const int32_t *y_b, Ctl *ctl)
{
    bool bad = false;
    for (int64_t b = blockIdx.y; b < n; b += gridDim.y) {
        const int32_t yb = y_b[b], mb = mate_b[b];
        for (int64_t a0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 8; a0 < na;
             a0 += (int64_t)gridDim.x * blockDim.x * 8) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int64_t a = a0 + e;
                if (a >= na) break;
                const int32_t s = y_a[a] + yb, kv = k[b * ldk + a];
                if (s > kv + 1 || (a == mb && s != kv)) bad = true;
            }
        }
    }
    if (bad) __hip_atomic_fetch_or(&ctl->err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// kMulti: many instances in one launch, `team` consecutive workgroups per
// instance, the instance's arguments in arr[blockIdx.x / team]; the barrier,
// lists and statistics of each instance involve only its own team.
template <int D>
struct SrcOf {
    using type = PointsSrc<D>;
    static __device__ type make(const LoopArgs &A) { return points_src<D>(A); }
};
template <>
struct SrcOf<0> {
    using type = MatrixSrc;
    static __device__ type make(const LoopArgs &A) { return MatrixSrc{A.k, A.ldk}; }
};
template <>
struct SrcOf<1> {
    using type = MatrixSrc8;
    static __device__ type make(const LoopArgs &A)
    {
        return MatrixSrc8{reinterpret_cast<const uint8_t *>(A.k), A.ldk};
    }
};

// kSrcD: 0 reads the rounded-cost matrix (1: stored as bytes); 2 or 3 computes it from points of
// that dimension (matrix-free). kFF: exact fast-forward through A.skip.
// kCopies: the rows are copies of the transport reduction (A.rmap, A.ymax).
// kTG: the workgroup's copy of the column duals is its slice of A.tpriv in
// global memory (only this workgroup touches it) instead of LDS.
template <bool kMulti, int kSrcD, bool kFF, bool kCopies = false, bool kTG = false>
__global__ void __launch_bounds__(kLoopThreads)
phase_loop_kernel(LoopArgs A0, const LoopArgs *__restrict__ arr, int team, int32_t *y_base)
{
    // the fast-forward's slack tracking costs registers: shallower prefetch
    constexpr int kScanAhead = kFF ? 4 : SrcOf<kSrcD>::type::kAhead;
    // the instance's arguments stay where they are (kernel arguments, or the
    // array in global memory), read through the scalar cache when needed
    const LoopArgs &A = kMulti ? arr[blockIdx.x / team] : A0;
    int32_t *const y_b = kMulti ? y_base + A.y_off : A.y_b;
    const typename SrcOf<kSrcD>::type src = SrcOf<kSrcD>::make(A);
    // rows beyond 17 bits come with columns beyond LDS (n_a >= n), so the
    // LDS instantiations keep the 17-bit packing as constants
    const RowPack P = row_pack(kTG ? A.wide : 0);
    // workgroups of this instance, and this workgroup's rank among them
    uint32_t nwg = kMulti ? (uint32_t)team : gridDim.x;
    uint32_t wg = kMulti ? blockIdx.x % (uint32_t)team : blockIdx.x;
    if (!kMulti && A0.gated) {
        // Plain launch: the workgroups that are resident take tickets; the
        // grid's last ticket, or a workgroup that waited kGateSpin polls for
        // the rest, closes the gate at the number of tickets handed out so
        // far. Those ticket holders run the loop as workgroups 0 .. nwg - 1
        // (all of them resident, so every round barrier completes); a later
        // workgroup leaves without touching any state. Which workgroups serve
        // which rows does not change the result.
        __shared__ uint32_t s_gate[2];
        if (threadIdx.x == 0) {
            Ctl *c = A0.ctl;
            const uint32_t cap = A0.gate_cap > 0 ? min((uint32_t)A0.gate_cap, gridDim.x) : gridDim.x;
            const uint32_t t = __hip_atomic_fetch_add(&c->gate_count, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (t + 1u == cap) {
                uint32_t expected = 0u;
                __hip_atomic_compare_exchange_strong(&c->gate, &expected, kGateClosed | cap,
                                                     __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
            }
            uint32_t g = ld_agent(&c->gate);
            for (int spins = 0; g == 0u; ++spins) {
                if (spins >= kGateSpin) {
                    const uint32_t got = ld_agent(&c->gate_count);
                    uint32_t expected = 0u;
                    __hip_atomic_compare_exchange_strong(&c->gate, &expected,
                                                         kGateClosed | min(got, cap),
                                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                }
                __builtin_amdgcn_s_sleep(2);
                g = ld_agent(&c->gate);
            }
            s_gate[0] = t;
            s_gate[1] = g & ~kGateClosed;
        }
        __syncthreads();
        wg = s_gate[0];
        nwg = s_gate[1];
        if (wg >= nwg) return;
        // every wave serves at most 64 rows of B'
        if ((int64_t)nwg * (kLoopThreads / kWave) * kWave < (int64_t)A0.n) {
            if (threadIdx.x == 0)
                __hip_atomic_fetch_or(&A0.ctl->err, 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
    }
    extern __shared__ __align__(16) uint16_t t_smem[];
    uint16_t *const t_lds = kTG ? A.tpriv + (int64_t)blockIdx.x * A.n_pad : t_smem;
    __shared__ uint32_t s_cnt_l, s_cnt_f, s_lose, s_nnext;
    __shared__ uint32_t s_base_l, s_base_f, s_ltot, s_over, s_abort;
    __shared__ unsigned long long s_scan, s_pend_scan;
    __shared__ int64_t s_pend_p;
    // per group: list lengths of the phase so far, last round's new taken
    // columns (start, count, prefix over groups), free-list prefix
    __shared__ uint32_t s_lcum[kMaxGroups], s_fcum[kMaxGroups], s_lstart[kMaxGroups],
        s_lnew[kMaxGroups], s_lpre[kMaxGroups], s_fpre[kMaxGroups];
    // team mode: best hit position of each team's row, by round parity
    __shared__ int s_best[2][kLoopThreads / kWave];
    __shared__ int s_mn[kLoopThreads / kWave];  // team mode: smallest k + t of a row's scan
    // regrouping into teams within a phase: rows still looking (by round
    // parity), slot of the next row handed over, the rows' scan states
    __shared__ uint32_t s_nact[2], s_kact;
    __shared__ int4 s_act[kLoopThreads / kWave / 2];

    const int lane = threadIdx.x & (kWave - 1);
    const int wpg = blockDim.x / kWave;
    const uint32_t W = nwg * wpg;
    const uint32_t gw = wg * wpg + threadIdx.x / kWave;
    const bool leader = wg == 0 && threadIdx.x == 0;
    Ctl *ctl = A.ctl;
    const int n = A.n;     // rows, |B|
    const int na = A.n_a;  // columns, |A| >= |B| (Section 3.3)

    const int G = A.groups;
    const int grp = (int)(wg % (uint32_t)G);
    const int64_t cap = A.list_cap;  // entries per group region of a list

    for (int i = threadIdx.x; i < A.n_pad; i += blockDim.x) t_lds[i] = A.t[i];
    uint32_t n_i = ld_agent(&ctl->free0);  // |B'| of the current phase
    if (threadIdx.x == 0) {
        s_cnt_l = s_cnt_f = s_lose = 0;
        s_abort = 0;
        s_scan = 0;
        s_pend_scan = 0;
        s_nact[0] = s_nact[1] = 0;
        s_kact = 0;
    }
    if (threadIdx.x < kMaxGroups) {
        // the first free list is one region (group 0)
        s_fpre[threadIdx.x] = threadIdx.x == 0 ? 0u : n_i;
        s_lcum[threadIdx.x] = s_fcum[threadIdx.x] = 0;
    }
    __syncthreads();

    // List entries written in phase p carry tag0 + p + 1; the free list of
    // the first phase carries tag0.
    const uint32_t tag0 = ld_agent(&ctl->tag_last) + 1u;
    uint32_t r = 0;                        // id of the last round (keys carry it)
    int64_t p = 0;                         // phase index within this launch
    // statistics, kept by the leader
    int64_t st_rounds = 0, st_max_rounds = 0, st_sum_free = 0;
    // Columns taken in the last round of the previous phase (list pend_L,
    // tag pend_tag, group layout still in s_lpre / s_lstart): their t is
    // raised when the next phase starts, so those reads overlap the reads of
    // the next free list, or when the loop ends.
    uint32_t pend = 0, pend_tag = 0;
    const unsigned long long *pend_L = nullptr;
    // entries examined in the last finished phase (s_pend_scan, phase
    // s_pend_p), added to the totals by thread 0 after a later arrival
    auto flush_scan = [&]() {
        const unsigned long long sc = s_pend_scan;
        if (sc) {
            add_agent(&ctl->scanned, sc);
            if (A.trace && s_pend_p < kTraceCap) add_agent(&A.trace[4 * s_pend_p + 2], (int64_t)sc);
            s_pend_scan = 0;
        }
    };
    auto apply_pending = [&]() {
        for (uint32_t i = threadIdx.x; i < pend; i += blockDim.x) {
            const int j = group_of(s_lpre, G, i);
            const int32_t a =
                take_entry(pend_L + j * cap + s_lstart[j] + (i - s_lpre[j]), pend_tag, na, &ctl->err);
            t_lds[a] = grown_t(t_lds[a], &ctl->err);
        }
        pend = 0;
    };
    for (;;) {
        if ((int64_t)n_i <= A.T) break;
        if (A.max_phases > 0 && p >= A.max_phases) {
            if (leader) ctl->status = 1;
            break;
        }
        // (r and p are the same in every workgroup, so all leave together)
        if (A.switch_round > 0 && p > 0 && r >= A.switch_round) {
            if (leader) ctl->status = 3;
            break;
        }
        // the watchdog: no run of the method needs more phases than this
        // bound (Lemma 3.2 with eq. (4)), so reaching it means the state
        // given to the loop was not one the method can reach
        if (A.phase_bound > 0 && p >= A.phase_bound) {
            if (leader) ctl->status = 2;
            break;
        }
        if (r >= P.round_limit) {
            if (leader) __hip_atomic_fetch_or(&ctl->err, 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        if (leader) {
            st_sum_free += n_i;
            if (A.trace && p < kTraceCap) A.trace[4 * p] = n_i;
            if (A.trace && p + 1 < kTraceCap)
                for (int i = 0; i < 4; ++i) st_agent(&A.trace[4 * (p + 1) + i], (int64_t)0);
        }
        const uint32_t tag = tag0 + (uint32_t)(p + 1);  // entries written in this phase
        const unsigned long long *Fc = A.F[p & 1];
        unsigned long long *Fn = A.F[(p + 1) & 1];
        unsigned long long *Lc = A.L[p & 1];
        uint32_t lcount = 0;  // length of the taken list after the last finished round
        uint32_t l_new = 0;   // columns taken in the last finished round
        int64_t phase_rounds = 0;

        // Slot mode (R = 1): slot s of this wave is entry gw + s*W of B' and
        // lane s holds its state. Team mode (|B'| <= W/2): R waves of a
        // workgroup (R a power of two, R <= W / |B'|, R <= 16) share one row,
        // entry `team`, and lane 0 of each of them holds its state.
        int R = 1;
        if (2 * n_i <= W) {
            const uint32_t q = W / n_i;
            R = q >= 16 ? 16 : (q >= 8 ? 8 : (q >= 4 ? 4 : 2));
        }
        // wave-uniform values, kept in scalar registers
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        int team_local = wv / R, k_rank = wv % R;
        const uint32_t team_id = wg * (uint32_t)(wpg / R) + (uint32_t)team_local;
        const uint32_t nslots = R == 1 ? (gw < n_i ? (n_i - gw + W - 1) / W : 0u)
                                       : (team_id < n_i ? 1u : 0u);
        if (threadIdx.x < 2 * (kLoopThreads / kWave))
            (&s_best[0][0])[threadIdx.x] = kNoHit;
        if (threadIdx.x < kLoopThreads / kWave) s_mn[threadIdx.x] = kNoHit;
        if (threadIdx.x < 2) s_nact[threadIdx.x] = 0;
        int32_t s_b = -1, s_yb = 0, s_pos = 0, s_a = 0, s_rb = 0;
        uint32_t s_skip = 0;
        unsigned long long s_key = 0;
        // this slot's entry of B' is loaded first, then the previous phase's
        // last taken columns; the two sets of reads are in flight together
        const unsigned long long *f_at = nullptr;
        unsigned long long f_val = 0;
        if ((uint32_t)lane < nslots) {
            const uint32_t e = R == 1 ? gw + (uint32_t)lane * W : team_id;
            const int j = group_of(s_fpre, G, e);
            f_at = Fc + j * cap + (e - s_fpre[j]);
            f_val = ld_agent(f_at);
        }
        apply_pending();
        __syncthreads();  // t of those columns and the team scratch are set
        if ((uint32_t)lane < nslots) {
            const uint32_t fv = take_raw_from(f_at, f_val, tag0 + (uint32_t)p, &ctl->err);
            s_b = min((int32_t)(fv & P.mask), n - 1);
            s_yb = (int32_t)(fv >> P.rb);
            if constexpr (kCopies) {
                // a free copy takes the largest dual of its point's copies
                // (every y(b) update of the last phase is in ymax by now)
                s_rb = A.rmap[s_b];
                const int32_t top = top_before(ld_agent(A.ymax + s_rb), p);
                if (top > s_yb) {
                    s_yb = top;
                    st_agent(y_b + s_b, top);
                }
            }
            if (kFF && A.skip) s_skip = ld_agent(A.skip + s_b);
        }
        // rows that cannot find a column this phase are exhausted without a scan
        const unsigned long long pre = __ballot((uint32_t)lane < nslots && s_skip > 0u);
        unsigned long long active = __ballot((uint32_t)lane < nslots) & ~pre;
        unsigned long long wave_scan = 0;
        bool first_round = true;

        for (;;) {
            r += 1;
            if (l_new) {
                // The rows of this wave that proposed: won (matched in M') or
                // lost (resume one position after the column). The keys are
                // final since the barrier; their loads go out first so that
                // they overlap the taken-list reads below.
                bool mine = (active >> lane) & 1ull;
                const unsigned long long k_now = mine ? ld_agent(A.key + s_a) : 0ull;
                // Columns taken in the previous round: marked for the rest of
                // the phase, t raised now (step (III a)).
                for (uint32_t i = threadIdx.x; i < l_new; i += blockDim.x) {
                    const int j = group_of(s_lpre, G, i);
                    const int32_t a =
                        take_entry(Lc + j * cap + s_lstart[j] + (i - s_lpre[j]), tag, na, &ctl->err);
                    t_lds[a] = (uint16_t)(grown_t(t_lds[a], &ctl->err) | kTaken);
                }
                if (mine) {
                    if (k_now == s_key) mine = false;
                    else s_pos += 1;
                }
                active = __ballot(mine);
                // rows of this workgroup still looking: a slot lane each, or
                // one per team (its first wave counts it)
                // (not for the copies of the transport reduction: a copy that
                // lost finds the next copy of the same column right after it,
                // so its scans stay short and teams only add overhead)
                constexpr bool kRegroup = !kCopies;
                const bool counts = R == 1 ? (active != 0ull) : (k_rank == 0 && (active & 1ull));
                if (kRegroup && R < 16 && lane == 0 && counts)
                    atomicAdd(&s_nact[r & 1], R == 1 ? (uint32_t)__popcll(active) : 1u);
                __syncthreads();
                if (kRegroup && R < 16) {
                    // Once the workgroup's rows still looking fit in half its
                    // waves per team (or, in slot mode, in half its waves),
                    // the phase continues with teams twice as large or more
                    // (the rows left are the ones whose scans run long): each
                    // row's state goes to LDS and R = 2..16 waves take it.
                    // Which waves scan a row does not change what they find.
                    const uint32_t nact = __builtin_amdgcn_readfirstlane(s_nact[r & 1]);
                    if (threadIdx.x == 0) s_nact[(r + 1) & 1] = 0;
                    if (nact > 0u && 2u * (uint32_t)R * nact <= (uint32_t)wpg) {
                        const bool mine_row = R == 1 ? ((active >> lane) & 1ull) != 0ull
                                                     : (k_rank == 0 && lane == 0 && (active & 1ull));
                        if (mine_row)
                            s_act[atomicAdd(&s_kact, 1u)] = make_int4(s_b, s_pos, s_yb, s_rb);
                        // a team that stopped looking left its last best hit
                        // in the buffer of this round's parity: start clean
                        if (threadIdx.x < 2 * (kLoopThreads / kWave))
                            (&s_best[0][0])[threadIdx.x] = kNoHit;
                        __syncthreads();
                        const uint32_t q = (uint32_t)wpg / nact;
                        R = q >= 16 ? 16 : (q >= 8 ? 8 : (q >= 4 ? 4 : 2));
                        team_local = wv / R;
                        k_rank = wv % R;
                        active = 0ull;
                        if ((uint32_t)team_local < nact) {
                            const int4 st = s_act[team_local];
                            s_b = st.x;
                            s_pos = st.y;
                            s_yb = st.z;
                            s_rb = st.w;
                            active = 1ull;
                        }
                        __syncthreads();
                        if (threadIdx.x == 0) s_kact = 0;
                    }
                }
            }
            unsigned long long s_old = 0;  // key a proposal of this lane's slot replaced
            bool proposed = false;
            uint32_t my_fv = kNoRow;       // row (and dual) this lane's slot puts on the next B'
            uint32_t n_prop = 0;
            // fast-forward: a full first-round scan that finds nothing records
            // the row's smallest slack
            const bool track = kFF && A.skip != nullptr && first_round;
            if (first_round && pre) {
                // exhausted as its scan from position 0 would be (extent na), (III b)
                const bool lead = R == 1 || k_rank == 0;
                if (lead) {
                    if ((pre >> lane) & 1ull) {
                        const int32_t y1 = grown_dual(s_yb, P.dual_max, &ctl->err);
                        st_agent(y_b + s_b, y1 < 0 ? s_yb : y1);
                        st_agent(A.skip + s_b, s_skip - 1u);
                        my_fv = y1 < 0 ? kNoRow : free_val(s_b, y1, P);
                    }
                    wave_scan += (unsigned long long)na * (unsigned long long)__popcll(pre);
                }
            }
            first_round = false;
            if (R > 1) {
                // team mode: every wave of the team scans its share of the row;
                // the team's first hit is the smallest position found
                int* best = &s_best[r & 1][team_local];
                if (active & 1ull) {
                    const SlotView v = slot_view(0, s_b, s_pos, s_yb, A.origin, na,
                                                 kCopies ? s_rb : s_b);
                    int mn = kNoHit;
                    const int j = team_scan(src, src.row(v.rb), t_lds, na, v.origin, v.S,
                                            v.yb - 1, k_rank, R, lane, best, track ? &mn : nullptr);
                    if (lane == 0 && j != kNoHit) atomicMin(best, j);
                    if (track) {
                        mn = wave_min(mn);
                        if (lane == 0) atomicMin(&s_mn[team_local], mn);
                    }
                }
                __syncthreads();
                if (active & 1ull) {
                    const SlotView v = slot_view(0, s_b, s_pos, s_yb, A.origin, na,
                                                 kCopies ? s_rb : s_b);
                    const int j = *best;
                    const int b = v.b, pos = v.pos, yb = v.yb;
                    const bool lead = k_rank == 0;
                    if (j != kNoHit) {
                        const int a = v.origin + j < na ? v.origin + j : v.origin + j - na;
                        const unsigned long long kn = make_key(r, b, yb, P);
                        if (lead) {
                            wave_scan += (unsigned long long)(j - pos + 1);
                            if (lane == 0) {
                                s_old = __hip_atomic_fetch_max(A.key + a, kn, __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT);
                                proposed = true;
                            }
                            n_prop = 1;
                        }
                        if (lane == 0) {
                            s_pos = j;
                            s_a = a;
                            s_key = kn;
                        }
                    } else {
                        // b has no admissible untaken column: free in M', (III b).
                        if (lead) {
                            wave_scan += (unsigned long long)(na - pos);
                            if (lane == 0) {
                                const int32_t y1 = grown_dual(yb, P.dual_max, &ctl->err);
                                st_agent(y_b + b, y1 < 0 ? yb : y1);
                                if constexpr (kCopies) raise_top(A.ymax + v.rb, p, y1 < 0 ? yb : y1);
                                my_fv = y1 < 0 ? kNoRow : free_val(b, y1, P);
                                if (track) {
                                    const int slack = s_mn[team_local] - (yb - 1);
                                    if (slack >= 2)
                                        st_agent(A.skip + b, (uint32_t)min(slack - 1, 1 << 30));
                                }
                            }
                        }
                        active = 0ull;
                    }
                    // the other buffer is cleared for the next round; every wave
                    // read it in the previous round, before this round's barriers
                    if (lead && lane == 0) s_best[(r + 1) & 1][team_local] = kNoHit;
                }
            }
            // Slot mode: rows are taken a few at a time (kBatch) so that their
            // first chunks are loaded together.
            unsigned long long rem = R == 1 ? active : 0ull;
            while (rem) {
                int sl[SrcOf<kSrcD>::type::kBatch];
                uint4 kvq[SrcOf<kSrcD>::type::kBatch];
#pragma unroll
                for (int q = 0; q < SrcOf<kSrcD>::type::kBatch; ++q) {
                    sl[q] = -1;
                    kvq[q] = make_uint4(0u, 0u, 0u, 0u);
                    if (!rem) continue;
                    sl[q] = __builtin_ctzll(rem);
                    rem &= rem - 1;
                    const SlotView v = slot_view(sl[q], s_b, s_pos, s_yb, A.origin, na,
                                                 kCopies ? s_rb : s_b);
                    const int col0 = v.base + lane * 8;
                    if (col0 < v.S.hi(v.sg))
                        kvq[q] = src.chunk(src.row(v.rb), col0);
                }
#pragma unroll
                for (int q = 0; q < SrcOf<kSrcD>::type::kBatch; ++q) {
                    if (sl[q] < 0) continue;
                    const int s = sl[q];
                    const SlotView v = slot_view(s, s_b, s_pos, s_yb, A.origin, na,
                                                 kCopies ? s_rb : s_b);
                    const int b = v.b, pos = v.pos, yb = v.yb;
                    const int slo = v.S.lo(v.sg), shi = v.S.hi(v.sg);
                    const int col0 = v.base + lane * 8;
                    const uint4 tv = col0 < shi ? *reinterpret_cast<const uint4 *>(t_lds + col0)
                                                : make_uint4(0u, 0u, 0u, 0u);
                    Hit h{-1, -1};
                    int mn = kNoHit;
                    if (track && col0 < shi)
                        mn = min_sum_masked(kvq[q], tv, range_mask(col0, slo, shi));
                    const int a = chunk_hit(col0, kvq[q], tv, yb - 1, slo, shi);
                    if (a >= 0) h = hit_at(a, v.origin, na);
                    else if (slo < shi)
                        h = scan_from<kScanAhead>(src, src.row(v.rb), t_lds, na, v.origin, v.S, v.sg,
                                      v.base + kChunk, yb - 1, lane, track ? &mn : nullptr);
                    if (h.j >= 0) {
                        wave_scan += (unsigned long long)(h.j - pos + 1);
                        const unsigned long long kn = make_key(r, b, yb, P);
                        if (lane == s) {
                            // the slot's own lane proposes, so proposals of several
                            // slots are in flight together
                            s_old = __hip_atomic_fetch_max(A.key + h.a, kn, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
                            proposed = true;
                            s_pos = h.j;
                            s_a = h.a;
                            s_key = kn;
                        }
                        n_prop += 1;
                    } else {
                        // b has no admissible untaken column: free in M', (III b).
                        wave_scan += (unsigned long long)(na - pos);
                        const int slack = track ? wave_min(mn) - (yb - 1) : 0;
                        if (lane == s) {
                            const int32_t y1 = grown_dual(yb, P.dual_max, &ctl->err);
                            st_agent(y_b + b, y1 < 0 ? yb : y1);
                            if constexpr (kCopies) raise_top(A.ymax + v.rb, p, y1 < 0 ? yb : y1);
                            my_fv = y1 < 0 ? kNoRow : free_val(b, y1, P);
                            if (slack >= 2) st_agent(A.skip + b, (uint32_t)min(slack - 1, 1 << 30));
                        }
                        active &= ~(1ull << s);
                    }
                }
            }
            // The first proposal to a column in a round: the column is in M'
            // whoever wins it, so step (II) evicts its old mate (if any) and
            // the column joins this phase's taken list.
            int32_t my_l = -1;
            if (proposed && (uint32_t)(s_old >> (15 + P.rb)) < r) {
                my_l = s_a;
                if (s_old != 0ull) my_fv = key_free(s_old, P);
            }
            const unsigned long long bl = __ballot(my_l >= 0), bf = __ballot(my_fv != kNoRow);
            uint32_t off_l = 0, off_f = 0;
            if (lane == 0) {
                const uint32_t nl = (uint32_t)__popcll(bl), nf = (uint32_t)__popcll(bf);
                off_l = atomicAdd(&s_cnt_l, nl);
                off_f = atomicAdd(&s_cnt_f, nf);
                if (n_prop > nl) s_lose = 1;  // a proposal of this wave lost
            }
            off_l = __builtin_amdgcn_readfirstlane(off_l);
            off_f = __builtin_amdgcn_readfirstlane(off_f);
            // Stores another workgroup reads in the next phase (the largest
            // dual of a point's copies, skip counts) are complete before the
            // arrival. The plain loop's y(b) stores are read only after the
            // launch; they complete before the row's entry of the next free
            // list is written (below), so a later store to the same y(b),
            // which follows a read of that entry, cannot overtake them.
            constexpr bool kStoresBeforeArrival = kCopies || kFF || kMulti;
            if (kStoresBeforeArrival) wait_memory();
            __syncthreads();

            // Arrival: the returned word is the sum over the workgroups of this
            // group that arrived before this one, which places this
            // workgroup's entries in the group's list regions.
            const bool timed = A.rtime != nullptr && r <= (uint32_t)kRoundTimeCap;
            unsigned long long *words = A.words + (r % 3) * kMaxGroups * kWordStride;
            if (threadIdx.x < kWave) {
                const int64_t t_arrive = timed ? (int64_t)wall_clock64() : 0;
                // the words of round r + 1 were last read in round r - 2, which
                // every workgroup has left
                if (wg == 0) {
                    if (lane < G)
                        st_agent(A.words + ((r + 1) % 3) * kMaxGroups * kWordStride +
                                     lane * kWordStride,
                                 0ull);
                    wait_memory();
                }
                if (threadIdx.x == 0) {
                    const unsigned long long add = (1ull << kShiftArrive) |
                                                   ((unsigned long long)s_lose << kShiftLose) |
                                                   ((unsigned long long)s_cnt_f << kShiftFree) |
                                                   (unsigned long long)s_cnt_l;
                    s_cnt_l = s_cnt_f = s_lose = 0;
                    const unsigned long long o = __hip_atomic_fetch_add(
                        words + grp * kWordStride, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_base_l = s_lcum[grp] + (uint32_t)(o & kField);
                    s_base_f = s_fcum[grp] + (uint32_t)((o >> kShiftFree) & kField);
                    flush_scan();
                    // the last arrival of each group records its time (one
                    // atomic per group rather than per workgroup)
                    if (timed && (uint32_t)(o >> kShiftArrive) + 1u ==
                                     nwg / (uint32_t)G + ((uint32_t)grp < nwg % (uint32_t)G ? 1u : 0u))
                        __hip_atomic_fetch_max(&A.rtime[3 * (r - 1)], t_arrive, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            {
                const uint32_t bl0 = s_base_l, bf0 = s_base_f;
                if (!kStoresBeforeArrival && bf != 0ull) wait_memory();
                if (my_l >= 0)
                    st_agent(Lc + grp * cap + bl0 + off_l + lanes_below(bl), tagged(tag, my_l));
                if (my_fv != kNoRow)
                    st_agent(Fn + grp * cap + bf0 + off_f + lanes_below(bf),
                             tagged(tag, (int32_t)my_fv));
            }
            if (threadIdx.x < kWave) {
                // lane j < G polls the word of group j until every workgroup
                // arrived, or the bounded wait runs out
                unsigned long long v;
                const int64_t t_wait = (int64_t)wall_clock64();
                bool late = false;
                for (int spins = 0;; ++spins) {
                    v = lane < G ? ld_agent(words + lane * kWordStride) : 0ull;
                    if (wave_sum((uint32_t)(v >> kShiftArrive)) == nwg) break;
                    if ((spins & 63) == 1 &&
                        (int64_t)wall_clock64() - t_wait >
                            (A.barrier_ticks > 0 ? A.barrier_ticks : kBarrierTicks)) {
                        late = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                if (late) {
                    if (lane == 0) {
                        __hip_atomic_fetch_or(&ctl->err, 32, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                    }
                    v = 0ull;  // no lists are read after an abort
                }
                const uint32_t nl = (uint32_t)(v & kField);
                const uint32_t nf = (uint32_t)((v >> kShiftFree) & kField);
                const uint32_t lose = (uint32_t)((v >> kShiftLose) & 0x7FFull);
                const uint32_t lpre = wave_exclusive_scan(nl, lane);
                const uint32_t ltot = wave_sum(nl), losers = wave_sum(lose);
                uint32_t fc = 0u;
                if (lane < G) {
                    s_lnew[lane] = nl;
                    s_lpre[lane] = lpre;
                    s_lstart[lane] = s_lcum[lane];
                    s_lcum[lane] += nl;
                    fc = s_fcum[lane] + nf;
                    s_fcum[lane] = fc;
                }
                if (lane == 0) {
                    s_ltot = ltot;
                    s_over = losers == 0u;
                }
                if (losers == 0u) {
                    // the phase is over: the next free list is the group
                    // regions of Fn, in group order
                    const uint32_t fpre = wave_exclusive_scan(fc, lane);
                    const uint32_t ftot = wave_sum(fc);
                    if (lane < G) {
                        s_fpre[lane] = fpre;
                        s_fcum[lane] = 0;
                        s_lcum[lane] = 0;
                    }
                    if (lane == 0) s_nnext = ftot;
                }
                if (timed && leader) {
                    A.rtime[3 * (r - 1) + 1] = (int64_t)wall_clock64();
                    A.rtime[3 * (r - 1) + 2] = p;
                }
            }
            __syncthreads();
            if (s_abort) break;
            l_new = s_ltot;
            lcount += l_new;
            if (l_new) phase_rounds += 1;  // some proposal was made this round
            if (s_over) break;
        }
        if (s_abort) break;
        // The marks of the phase are cleared; the columns taken in its last
        // round (not marked) get their t raised later, see pend.
        pend = l_new;
        pend_tag = tag;
        pend_L = Lc;
        for (int i = threadIdx.x * 8; i < A.n_pad; i += blockDim.x * 8) {
            uint4 *q = reinterpret_cast<uint4 *>(t_lds + i);
            uint4 v = *q;
            v.x &= 0x7FFF7FFFu;
            v.y &= 0x7FFF7FFFu;
            v.z &= 0x7FFF7FFFu;
            v.w &= 0x7FFF7FFFu;
            *q = v;
        }
        // entries examined this phase, one atomic per workgroup
        if (lane == 0 && wave_scan) atomicAdd(&s_scan, wave_scan);
        __syncthreads();
        if (threadIdx.x == 0) {
            // added to the totals after this workgroup's next arrival: every
            // workgroup adds to the same two words, and a wave waits for its
            // own atomics to complete before it arrives
            s_pend_scan = s_scan;
            s_pend_p = p;
            s_scan = 0;
        }
        if (leader) {
            st_rounds += phase_rounds;
            if (phase_rounds > st_max_rounds) st_max_rounds = phase_rounds;
            if (A.trace && p < kTraceCap) {
                A.trace[4 * p + 1] = phase_rounds;
                A.trace[4 * p + 3] = lcount;
            }
        }
        n_i = s_nnext;
        p += 1;
    }
    if (threadIdx.x == 0) flush_scan();
    if (leader) {
        // after a phase every workgroup has read tag_last (before arriving)
        // (an aborted phase used tag0 + p + 1 as well)
        if (p > 0 || s_abort) ctl->tag_last = tag0 + (uint32_t)p + (s_abort ? 1u : 0u);
        ctl->phases = p;
        ctl->sum_free = st_sum_free;
        ctl->rounds = st_rounds;
        ctl->max_rounds = st_max_rounds;
        ctl->free_after = n_i;
    }
    // (after an abort the state is not used: the host reports the error)
    if (wg == 0 && !s_abort) {
        apply_pending();
        __syncthreads();
        for (int i = threadIdx.x; i < na; i += blockDim.x) A.t[i] = t_lds[i];
    }
}

// Clears the bits `mask` of the error word (all of them, or only the
// too-few-workgroups bit before a cooperative relaunch, keeping what the cost
// build reported).
__global__ void clear_err_kernel(Ctl *ctl, int32_t mask) { ctl->err &= ~mask; }

__global__ void fill64_kernel(int64_t *p, int64_t n, int64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Matching and duals from the per-column keys and t.
__global__ void decode_kernel(LoopArgs a, int32_t *mate_a, int32_t *mate_b, int32_t *y_a)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_a; i += gridDim.x * blockDim.x) {
        const unsigned long long kk = a.key[i];
        const int32_t m = kk ? key_row(kk, row_pack(a.wide)) : -1;
        mate_a[i] = m;
        if (m >= 0) mate_b[m] = i;
        y_a[i] = -(int32_t)a.t[i];
    }
}

constexpr int kCompleteThreads = 1024;

// The ascending list of the indices i < n with mate[i] < 0, by one workgroup
// of kCompleteThreads threads: tiles of kCompleteThreads consecutive indices
// (coalesced), kListTiles tiles' loads in flight at a time (every load is
// issued, past the end clamped to index n - 1, so that none waits behind a
// branch), a ballot per wave and an ordered prefix over the waves of the
// tiles. Returns the count.
constexpr int kListTiles = 16;
constexpr int kListWaves = kCompleteThreads / 64;

__device__ __forceinline__ int list_flags(const int32_t *__restrict__ mate, int n,
                                          int32_t *__restrict__ out, int *cnt)
{
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const unsigned long long below = (1ull << lane) - 1ull;
    int base = 0;
    for (int t0 = 0; t0 < n; t0 += kListTiles * kCompleteThreads) {
        int32_t v[kListTiles];
#pragma unroll
        for (int q = 0; q < kListTiles; ++q) {
            const int i = t0 + q * kCompleteThreads + tid;
            v[q] = mate[i < n ? i : n - 1];
        }
        bool f[kListTiles];
#pragma unroll
        for (int q = 0; q < kListTiles; ++q)
            f[q] = t0 + q * kCompleteThreads + tid < n && v[q] < 0;
        unsigned long long bal[kListTiles];
#pragma unroll
        for (int q = 0; q < kListTiles; ++q) {
            bal[q] = __ballot(f[q]);
            if (lane == 0) cnt[q * kListWaves + wv] = __popcll(bal[q]);
        }
        __syncthreads();
        if (wv == 0) {
            // exclusive prefix in index order (tile by tile, wave by wave
            // within a tile): kPer consecutive counts per lane, then a scan
            // over the lanes
            constexpr int kPer = kListTiles * kListWaves / kWave;
            static_assert(kPer * kWave == kListTiles * kListWaves, "whole counts per lane");
            int c[kPer];
            int own = 0;
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                c[e] = cnt[kPer * lane + e];
                own += c[e];
            }
            int run = own;
#pragma unroll
            for (int off = 1; off < kWave; off <<= 1) {
                const int v = __shfl_up(run, off);
                if (lane >= off) run += v;
            }
            int before = run - own;
#pragma unroll
            for (int e = 0; e < kPer; ++e) {
                cnt[kPer * lane + e] = before;
                before += c[e];
            }
            if (lane == kWave - 1) cnt[kListTiles * kListWaves] = run;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kListTiles; ++q)
            if (f[q])
                out[base + cnt[q * kListWaves + wv] + __popcll(bal[q] & below)] =
                    t0 + q * kCompleteThreads + tid;
        base += cnt[kListTiles * kListWaves];
        __syncthreads();
    }
    return base;
}

// Copies of the transport reduction: when the loop ends, every free copy
// takes the largest dual of its point's copies (as after each phase).
__global__ void raise_free_kernel(LoopArgs a, const int32_t *mate_b)
{
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < a.n; b += gridDim.x * blockDim.x)
        if (mate_b[b] < 0) {
            const int32_t top = (int32_t)(uint32_t)a.ymax[a.rmap[b]];
            if (top > a.y_b[b]) a.y_b[b] = top;
        }
}

// Completion (Section 2.1): the i-th free b (ascending) takes the i-th free a.
// A loop stopped by max_phases is left as it is (a state to resume from).
__global__ void __launch_bounds__(kCompleteThreads)
complete_kernel(int n, int n_a, int32_t *mate_a, int32_t *mate_b, int32_t *scratch,
                int32_t complete, const Ctl *ctl)
{
    __shared__ int cnt[kCompleteThreads];
    // read first: their latency hides behind the lists
    const int32_t stopped = ctl->status, err = ctl->err;
    if (err & kErrLoop) {
        // the loop failed: the outputs are marked invalid (every vertex
        // free); the host reports the error
        for (int i = threadIdx.x; i < n; i += kCompleteThreads) mate_b[i] = -1;
        for (int i = threadIdx.x; i < n_a; i += kCompleteThreads) mate_a[i] = -1;
        return;
    }
    const int nb = list_flags(mate_b, n, scratch, cnt);
    const int na = list_flags(mate_a, n_a, scratch + n, cnt);
    // a loop stopped early (max_phases, the watchdog, or too few workgroups
    // resident, when nothing ran) keeps its state for a resume
    if (!complete || stopped || err) return;
    const int m = min(nb, na);
    for (int i = threadIdx.x; i < m; i += kCompleteThreads) {
        const int b = scratch[i], a = scratch[n + i];
        mate_b[b] = a;
        mate_a[a] = b;
    }
}

constexpr int kFinalizeThreads = 256;

// Per-block partial sums, in a fixed order, of k and of the cost over the
// matching (deterministic: the host adds the partials in block order).
__global__ void __launch_bounds__(kFinalizeThreads)
finalize_kernel(int64_t n, const int32_t *mate_b, const int16_t *k, int64_t ldk, int cost_kind,
                const float *C, int64_t ldc, const float *X, const float *Y, int32_t d,
                long long *part_k, double *part_c, const float *m_dev, double eps,
                const float *th, int k8)
{
    // costs on the fly: the cost build's rounding of each matched pair
    int K = 0;
    float inv = 0.0f, delta = 0.0f;
    if (!k && m_dev) {
        const float mf = *m_dev;
        K = (mf > 0.0f) ? (int32_t)floor(1.0 / eps) : 0;
        inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * eps)) : 0.0f;
        delta = classify_margin(K);
    }
    __shared__ long long sk[kFinalizeThreads];
    __shared__ double sc[kFinalizeThreads];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = min<int64_t>(n, blockIdx.x * per), hi = min<int64_t>(n, lo + per);
    long long ks = 0;
    double cs = 0.0;
    for (int64_t b = lo + threadIdx.x; b < hi; b += kFinalizeThreads) {
        const int32_t a = mate_b[b];
        if (a < 0) continue;
        if (k) {
            ks += k8 ? reinterpret_cast<const uint8_t *>(k)[b * ldk + a] : k[b * ldk + a];
        } else if (m_dev) {
            const float sq = sqdist<0>(X + b * d, Y + (int64_t)a * d, d);
            bool ok;
            int g = fast_k(sq, inv, delta, K, ok);
            if (!ok) g = refine_k(sq, g, K, th);
            ks += g;
        }
        if (cost_kind == 1) {
            cs = __dadd_rn(cs, (double)C[b * ldc + a]);
        } else if (cost_kind == 2 || cost_kind == 3) {
            // squared Euclidean (the host divides by m) or Euclidean (by sqrt m)
            double s = 0.0;
            for (int j = 0; j < d; ++j) {
                const double t = __dsub_rn((double)X[b * d + j], (double)Y[(int64_t)a * d + j]);
                s = __dadd_rn(s, __dmul_rn(t, t));
            }
            cs = __dadd_rn(cs, cost_kind == 3 ? sqrt(s) : s);
        } else if (cost_kind == 4) {
            // half the L1 distance of the vectors normalised to sum 1
            double sx = 0.0, sy = 0.0, s = 0.0;
            for (int j = 0; j < d; ++j) {
                sx = __dadd_rn(sx, (double)X[b * d + j]);
                sy = __dadd_rn(sy, (double)Y[(int64_t)a * d + j]);
            }
            for (int j = 0; j < d; ++j)
                s = __dadd_rn(s, fabs(__dsub_rn((double)X[b * d + j] / sx,
                                                (double)Y[(int64_t)a * d + j] / sy)));
            cs = __dadd_rn(cs, 0.5 * s);
        }
    }
    sk[threadIdx.x] = ks;
    sc[threadIdx.x] = cs;
    __syncthreads();
    for (int off = kFinalizeThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sk[threadIdx.x] += sk[threadIdx.x + off];
            sc[threadIdx.x] = __dadd_rn(sc[threadIdx.x], sc[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part_k[blockIdx.x] = sk[0];
        part_c[blockIdx.x] = sc[0];
    }
}

// Batched teams, set-up of every instance: the cold start of the init
// kernel plus the reset of its control block and round words.
__global__ void team_init_kernel(TeamArgs T)
{
    const LoopArgs a = T.loops[blockIdx.y];
    int32_t *y_b = T.y_b + a.y_off;
    const uint32_t tag0 = a.ctl->tag_last + 1u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_pad; i += gridDim.x * blockDim.x) {
        if (i < a.n) {
            a.key[i] = 0ull;
            a.t[i] = 0;
            y_b[i] = 1;
            a.F[0][i] = tagged(tag0, (int32_t)free_val(i, 1, row_pack(a.wide)));
            if (a.skip) a.skip[i] = 0u;
        } else {
            a.t[i] = 0;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Ctl *c = a.ctl;
        for (int i = 0; i < 3 * kMaxGroups; ++i) a.words[i * kWordStride] = 0ull;
        c->free0 = (uint32_t)a.n;
        c->scanned = 0;
        c->status = 0;
        c->err = 0;
        c->phases = c->sum_free = c->rounds = c->max_rounds = 0;
        c->free_after = 0;
    }
}

// Batched teams, one workgroup per instance after the loop: matching and
// duals from the keys and t, the completion (Section 2.1: the i-th free b in
// ascending order takes the i-th free a), and the instance's statistics
// (fixed-order reductions, binary64 cost).
__global__ void __launch_bounds__(kCompleteThreads) team_finish_kernel(TeamArgs T)
{
    __shared__ int cnt[kCompleteThreads];
    __shared__ long long red_k[kCompleteThreads];
    __shared__ double red_c[kCompleteThreads];
    const int inst = blockIdx.x;
    const int tid = threadIdx.x;
    const LoopArgs a = T.loops[inst];
    const int n = a.n;
    const int64_t off = T.pt_off[inst];
    int32_t *ma = T.mate_a + off, *mb = T.mate_b + off, *ya = T.y_a + off;
    for (int i = tid; i < n; i += kCompleteThreads) mb[i] = -1;
    __syncthreads();
    for (int i = tid; i < n; i += kCompleteThreads) {
        const unsigned long long kk = a.key[i];
        const int32_t b = kk ? key_row(kk, row_pack(a.wide)) : -1;
        ma[i] = b;
        if (b >= 0) mb[b] = i;
        ya[i] = -(int32_t)a.t[i];
    }
    __syncthreads();
    int32_t *sc = T.scratch + 2 * off;
    const int nb = list_flags(mb, n, sc, cnt);
    const int na = list_flags(ma, n, sc + n, cnt);
    // no completion after the watchdog stopped the loop or the loop failed
    if (T.complete && a.ctl->status != 2 && !(a.ctl->err & kErrLoop)) {
        const int m = min(nb, na);
        for (int i = tid; i < m; i += kCompleteThreads) {
            mb[sc[i]] = sc[n + i];
            ma[sc[n + i]] = sc[i];
        }
    }
    __syncthreads();
    const float *X = T.X + off * T.d, *Y = T.Y + off * T.d;
    long long ks = 0;
    double cs = 0.0;
    for (int b = tid; b < n; b += kCompleteThreads) {
        const int32_t c = mb[b];
        if (c < 0) continue;
        ks += a.k[(int64_t)b * a.ldk + c];
        double s = 0.0;
        for (int q = 0; q < T.d; ++q) {
            const double dq =
                __dsub_rn((double)X[(int64_t)b * T.d + q], (double)Y[(int64_t)c * T.d + q]);
            s = __dadd_rn(s, __dmul_rn(dq, dq));
        }
        cs = __dadd_rn(cs, s);
    }
    red_k[tid] = ks;
    red_c[tid] = cs;
    __syncthreads();
    for (int o = kCompleteThreads / 2; o > 0; o >>= 1) {
        if (tid < o) {
            red_k[tid] += red_k[tid + o];
            red_c[tid] = __dadd_rn(red_c[tid], red_c[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const Ctl &c = *a.ctl;
        InstanceStats &st = T.stats[inst];
        const float m = T.m[inst];
        st.phases = c.phases;
        st.sum_free = c.sum_free;
        st.rounds = c.rounds;
        st.max_rounds = c.max_rounds;
        st.scanned = (int64_t)c.scanned;
        st.matched_in_phases = n - c.free_after;
        st.completed_pairs = T.complete ? c.free_after : 0;
        st.sum_k = red_k[0];
        st.threshold = a.T;
        st.status = c.status ? 1 : 0;
        st.kmax = m > 0.0f ? (int32_t)floor(1.0 / T.eps) : 0;
        st.cost_scale = (double)m;
        st.cost = m > 0.0f ? red_c[0] / (double)m : 0.0;
        if (c.status == 2) {
            st.status = -4;  // PROT_E_PHASE_BOUND
            __hip_atomic_fetch_or(T.err, 256, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (c.err & kErrLoop) {
            st.status = -6;
            __hip_atomic_fetch_or(T.err, c.err & kErrLoop, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

inline unsigned blocks_for(int64_t n, int threads)
{
    int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

}  // namespace

hipError_t launch_init(const LoopArgs &a, int32_t warm, const int32_t *mate_a,
                       int32_t *mate_b, const int32_t *y_a, hipStream_t s)
{
    // a warm start counts its free rows with atomics on a word reset first
    if (warm) hipLaunchKernelGGL(loop_reset_kernel, dim3(1), dim3(1), 0, s, a);
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(a.n_pad > a.n ? a.n_pad : a.n, 256)), dim3(256),
                       0, s, a, warm,
                       mate_a, mate_b, y_a);
    return hipGetLastError();
}

hipError_t launch_clear_err(Ctl *ctl, hipStream_t s, int32_t mask)
{
    hipLaunchKernelGGL(clear_err_kernel, dim3(1), dim3(1), 0, s, ctl, mask);
    return hipGetLastError();
}

hipError_t launch_check_state(int64_t n, int64_t na, const int32_t *mate_a,
                              const int32_t *mate_b, const int32_t *y_a, const int32_t *y_b,
                              int32_t ybound, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(check_state_kernel, dim3(blocks_for(na, 256)), dim3(256), 0, s, n, na,
                       mate_a, mate_b, y_a, y_b, ybound, ctl);
    return hipGetLastError();
}

hipError_t launch_check_feasible(const int16_t *k, int64_t ldk, int64_t n, int64_t na,
                                 const int32_t *mate_b, const int32_t *y_a, const int32_t *y_b,
                                 Ctl *ctl, hipStream_t s)
{
    const unsigned gx = blocks_for((na + 7) / 8, 256);
    const unsigned gy = (unsigned)(n < 4096 ? (n < 1 ? 1 : n) : 4096);
    hipLaunchKernelGGL(check_feasible_kernel, dim3(gx, gy), dim3(256), 0, s, k, ldk, n, na,
                       mate_b, y_a, y_b, ctl);
    return hipGetLastError();
}

hipError_t launch_clear_times(int64_t *rtime, hipStream_t s)
{
    hipLaunchKernelGGL(fill64_kernel, dim3(256), dim3(256), 0, s, rtime,
                       (int64_t)3 * kRoundTimeCap, (int64_t)0);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    hipLaunchKernelGGL(fill64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, (int64_t *)p, n,
                       (int64_t)v);
    return hipGetLastError();
}

hipError_t loop_grid(int32_t n_pad, int wgs_per_cu, int *grid_max)
{
    const size_t lds = (size_t)n_pad * sizeof(uint16_t);
    hipError_t e = hipSuccess;
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void *)phase_loop_kernel<false, 0, false>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, phase_loop_kernel<false, 0, false>,
                                                     kLoopThreads, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (per_cu > wgs_per_cu) per_cu = wgs_per_cu;
    *grid_max = per_cu * cus;
    // arrivals and losing workgroups are 11-bit fields of the round word
    if (*grid_max > 2047) *grid_max = 2047;
    return hipSuccess;
}

// Occupancy-limited grid of the loop with its column duals in global memory.
hipError_t loop_grid_tg(int wgs_per_cu, int *grid_max)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, phase_loop_kernel<false, 0, false, false, true>, kLoopThreads, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    if (per_cu > wgs_per_cu) per_cu = wgs_per_cu;
    *grid_max = per_cu * cus;
    if (*grid_max > 2047) *grid_max = 2047;
    return hipSuccess;
}

hipError_t launch_loop(const LoopArgs &a, int grid, hipStream_t s, hipEvent_t ev_start,
                       hipEvent_t ev_stop)
{
    LoopArgs copy = a;
    const LoopArgs *none = nullptr;
    int team = 1;
    int32_t *no_base = nullptr;
    void *args[] = {&copy, &none, &team, &no_base};
    const size_t lds = a.tpriv ? 0 : (size_t)a.n_pad * sizeof(uint16_t);
    const void *fn =
        a.tpriv ? (a.rmap      ? (const void *)phase_loop_kernel<false, 0, false, true, true>
                   : a.pd == 2 ? (const void *)phase_loop_kernel<false, 2, false, false, true>
                   : a.pd == 3 ? (const void *)phase_loop_kernel<false, 3, false, false, true>
                   : a.k8      ? (const void *)phase_loop_kernel<false, 1, false, false, true>
                               : (const void *)phase_loop_kernel<false, 0, false, false, true>)
        : a.rmap    ? (const void *)phase_loop_kernel<false, 0, false, true>
        : a.pd == 2 ? (const void *)phase_loop_kernel<false, 2, false>
        : a.pd == 3 ? (const void *)phase_loop_kernel<false, 3, false>
        : a.k8      ? (const void *)phase_loop_kernel<false, 1, false>
                    : (const void *)phase_loop_kernel<false, 0, false>;
    if (!a.tpriv && (a.pd || a.rmap || a.k8) && lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)lds);
        if (e != hipSuccess) return e;
    }
    // a plain launch (a cooperative one costs ~20 us more here); the gate at
    // the kernel's start makes it safe when not every workgroup is resident.
    // The events take the launch's own start and end (events recorded on
    // the stream around it would each hold the next launch back ~6 us).
    if (a.gated)
        return hipExtLaunchKernel(fn, dim3(grid), dim3(kLoopThreads), args, lds, s, ev_start,
                                  ev_stop, 0);
    hipError_t e = ev_start ? hipEventRecord(ev_start, s) : hipSuccess;
    if (e == hipSuccess)
        e = hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kLoopThreads), args, (unsigned)lds, s);
    if (e == hipSuccess && ev_stop) e = hipEventRecord(ev_stop, s);
    return e;
}

hipError_t loop_grid_multi(int32_t n_pad_max, int wgs_per_cu, int *grid_max)
{
    const size_t lds = (size_t)n_pad_max * sizeof(uint16_t);
    hipError_t e = hipSuccess;
    if (lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void *)phase_loop_kernel<true, 0, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0, dev = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, phase_loop_kernel<true, 0, true>,
                                                     kLoopThreads, lds);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    if (per_cu > wgs_per_cu) per_cu = wgs_per_cu;
    *grid_max = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_team_init(const TeamArgs &t, int32_t n_pad_max, hipStream_t s)
{
    if (t.batch > 0)
        hipLaunchKernelGGL(team_init_kernel, dim3(blocks_for(n_pad_max, 256), (unsigned)t.batch),
                           dim3(256), 0, s, t);
    return hipGetLastError();
}

hipError_t launch_loop_multi(const LoopArgs *arr, int count, int team, int32_t n_pad_max,
                             int32_t *y_base, hipStream_t s)
{
    LoopArgs none{};
    void *args[] = {&none, &arr, &team, &y_base};
    const size_t lds = (size_t)n_pad_max * sizeof(uint16_t);
    return hipLaunchCooperativeKernel((const void *)phase_loop_kernel<true, 0, true>,
                                      dim3((unsigned)(count * team)), dim3(kLoopThreads), args,
                                      (unsigned)lds, s);
}

hipError_t launch_team_finish(const TeamArgs &t, hipStream_t s)
{
    if (t.batch > 0)
        hipLaunchKernelGGL(team_finish_kernel, dim3((unsigned)t.batch), dim3(kCompleteThreads), 0,
                           s, t);
    return hipGetLastError();
}

hipError_t launch_finish(const LoopArgs &a, int32_t warm, int32_t complete, int32_t *mate_a,
                         int32_t *mate_b, int32_t *y_a, int32_t *scratch, hipStream_t s)
{
    // a cold start's init already set mate_b to -1
    if (warm)
        hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, mate_b,
                           (int64_t)a.n, -1);
    hipLaunchKernelGGL(decode_kernel, dim3(blocks_for(a.n_a, 256)), dim3(256), 0, s, a, mate_a,
                       mate_b, y_a);
    if (a.rmap)
        hipLaunchKernelGGL(raise_free_kernel, dim3(blocks_for(a.n, 256)), dim3(256), 0, s, a,
                           mate_b);
    hipLaunchKernelGGL(complete_kernel, dim3(1), dim3(kCompleteThreads), 0, s, a.n, a.n_a,
                       mate_a, mate_b, scratch, complete, a.ctl);
    return hipGetLastError();
}

hipError_t launch_finalize(int64_t n, const int32_t *mate_b, const int16_t *k, int64_t ldk,
                           int cost_kind, const float *C, int64_t ldc, const float *X,
                           const float *Y, int32_t d, long long *part_k, double *part_c,
                           hipStream_t s, const float *m_dev, double eps, const float *th,
                           int k8)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(kFinalizeBlocks), dim3(kFinalizeThreads), 0, s, n,
                       mate_b, k, ldk, cost_kind, C, ldc, X, Y, d, part_k, part_c, m_dev, eps,
                       th, k8);
    return hipGetLastError();
}

}  // namespace prot
