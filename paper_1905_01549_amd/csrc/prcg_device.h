// Device helpers shared by the libprcg kernels: deterministic reductions,
// the XCD-aware split of rows over workgroups and the sparse row products.
#pragma once

#include "prcg_common.h"

namespace prcg {

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum over the 64 lanes of a wavefront by a fixed butterfly; every lane ends
// with the same bits (each level adds the same two operands).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of NV values over a workgroup of NW wavefronts; every thread receives
// the totals.  The order of additions is fixed, so results are repeatable.
template <int NV, int NW = kWaves>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* NW * NV */)
{
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[w * NV + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = lds[i];
#pragma unroll
        for (int q = 1; q < NW; ++q) t += lds[q * NV + i];
        v[i] = t;
    }
    __syncthreads();
}

// Stage 2 of a reduction: the G per-workgroup partials of each of NV values
// are summed in one fixed order (G <= kMaxGrid).  Value i < N1 is read from
// P1[i * Gs + g], value i >= N1 from P2[(i - N1) * Gs + g] (two kernels may
// produce the partials of one reduction; the rows are 16-byte aligned).  The
// order: the partials are taken in pairs (2k, 2k + 1), read as one 16-byte
// load; lane t < kBlock owns the pairs k = t + kBlock j, j = 0 .. kChunks
// kChunkPairs - 1 (partials at or beyond G count as absent), in kChunks
// chunks of kChunkPairs consecutive j; each chunk's partials are added in
// order from 0.0, and the lane's sum is ((c_0 + c_1) + c_2) + c_3 over its
// chunk sums (an absent chunk adds 0.0); the kBlock lane sums go through
// block_sum.  Every thread receives the totals.
//
// ALL = false (kernels that reduce beside other work, kBlock threads):
// thread t is lane t and walks its chunks in order, loading two pairs per
// value at a time, to keep its register count down.  lds: kWaves * NV
// doubles.
// ALL = true (the one-workgroup stage-2 kernels, kStage2Block = 2 kBlock
// threads): threads t and t + kBlock take the chunks of lane t in turns
// (chunks 0 and 2, and 1 and 3), each chunk with all its loads issued before
// its first addition, so stage 2 costs one memory round trip up to
// G = 2 kBlock kChunkPairs partials and two beyond; chunks without a
// partial below G load nothing.  lds: kStage2Waves * NV doubles.
// (Measured on MI355X: a one-workgroup reduction is bound by its load
// instructions, so 16-byte loads halve its cost; 1024-thread workgroups are
// limited to 128 registers per thread and spilled.)  The bits are the same
// either way.
constexpr int kChunkPairs = 8;                                  // pairs per chunk
constexpr int kChunks = kMaxGrid / (2 * kBlock * kChunkPairs);  // chunks per lane
static_assert(kChunks == 4, "the lane sum adds four chunk sums");
constexpr int kStage2Block = 2 * kBlock;
constexpr int kStage2Waves = kStage2Block / 64;

// The pair k of row P (k < G / 2 rounded up), partials beyond G as 0.0; the
// load itself is clamped to the last pair, so it stays in bounds.
__device__ __forceinline__ double2 load_pair(const double* __restrict__ P, int k, int G)
{
    const int kc = min(k, (G - 1) >> 1);
    return reinterpret_cast<const double2*>(P)[kc];
}

// adds pair k's partials that lie below G to a
__device__ __forceinline__ double add_pair(double a, double2 v, int k, int G)
{
    a += 2 * k < G ? v.x : 0.0;
    a += 2 * k + 1 < G ? v.y : 0.0;
    return a;
}

// Whether chunk c of some lane holds a partial below G.
__device__ __forceinline__ bool chunk_used(int c, int G) { return 2 * kBlock * kChunkPairs * c < G; }

// Chunk c of lane `lane` for NV values: every load issued before the first
// addition (one memory round trip); sums from 0.0 in pair order.
template <int NV>
__device__ __forceinline__ void chunk_sum(const double* const (&P)[NV], int lane, int c, int G, double (&sum)[NV])
{
#pragma unroll
    for (int i = 0; i < NV; ++i) sum[i] = 0.0;
    if (!chunk_used(c, G)) return;
    double2 buf[NV][kChunkPairs];
#pragma unroll
    for (int j = 0; j < kChunkPairs; ++j) {
        const int k = lane + kBlock * (c * kChunkPairs + j);
#pragma unroll
        for (int i = 0; i < NV; ++i) buf[i][j] = load_pair(P[i], k, G);
    }
    // keep the scheduler from starting the sums before the last load
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
        for (int j = 0; j < kChunkPairs; ++j) sum[i] = add_pair(sum[i], buf[i][j], lane + kBlock * (c * kChunkPairs + j), G);
    }
}

template <int NV, int N1>
__device__ __forceinline__ void partial_rows(const double* __restrict__ P1, const double* __restrict__ P2, int Gs,
                                             const double* (&P)[NV])
{
#pragma unroll
    for (int i = 0; i < NV; ++i) P[i] = i < N1 ? P1 + (int64_t)i * Gs : P2 + (int64_t)(i - N1) * Gs;
}

template <int NV, int N1, bool ALL = false, int M>
__device__ __forceinline__ void reduce_partials_at(const double* __restrict__ P1, const double* __restrict__ P2, int G,
                                                   int Gs, double (&tot)[NV], double (&lds)[M])
{
    static_assert(M >= (ALL ? kStage2Waves : kWaves) * NV, "lds must hold one sum per wavefront and value");
    const double* P[NV];
    partial_rows<NV, N1>(P1, P2, Gs, P);
    double acc[NV];
    if constexpr (ALL) {
        __shared__ double odd[2][NV][kBlock];  // chunks 1 and 3 of each lane
        const int lane = threadIdx.x % kBlock;
        const int half = threadIdx.x / kBlock;  // uniform per wavefront
        double c0[NV], c1[NV];
        chunk_sum<NV>(P, lane, half, G, c0);
        chunk_sum<NV>(P, lane, half + 2, G, c1);
        if (half == 1) {
#pragma unroll
            for (int i = 0; i < NV; ++i) {
                odd[0][i][lane] = c0[i];
                odd[1][i][lane] = c1[i];
            }
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] = ((c0[i] + odd[0][i][lane]) + c1[i]) + odd[1][i][lane];
        } else {
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] = 0.0;
        }
        // every wavefront writes its sum; only the first kWaves (lanes
        // 0 .. kBlock - 1) are added
        block_sum<NV, kWaves>(acc, lds);
    } else {
        // chunk 0 two pairs per value at a time; the other chunks (only when
        // G exceeds chunk 0) one pair at a time, so that their accumulators
        // cost no registers beyond chunk 0's
        const int t = threadIdx.x;
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] = 0.0;
        for (int j0 = 0; j0 < kChunkPairs && 2 * kBlock * j0 < G; j0 += 2) {
            double2 buf[NV][2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
#pragma unroll
                for (int i = 0; i < NV; ++i) buf[i][j] = load_pair(P[i], t + kBlock * (j0 + j), G);
            }
#pragma unroll
            for (int i = 0; i < NV; ++i) {
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i] = add_pair(acc[i], buf[i][j], t + kBlock * (j0 + j), G);
            }
        }
        for (int c = 1; c < kChunks; ++c) {
            double cs[NV];
#pragma unroll
            for (int i = 0; i < NV; ++i) cs[i] = 0.0;
            for (int j = c * kChunkPairs; j < (c + 1) * kChunkPairs && 2 * kBlock * j < G; ++j) {
                double2 buf[NV];
#pragma unroll
                for (int i = 0; i < NV; ++i) buf[i] = load_pair(P[i], t + kBlock * j, G);
#pragma unroll
                for (int i = 0; i < NV; ++i) cs[i] = add_pair(cs[i], buf[i], t + kBlock * j, G);
            }
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[i] = acc[i] + cs[i];
        }
        block_sum<NV>(acc, lds);
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = acc[i];
}

// Stage 2 split over kWaves workgroups (grid kWaves, kWaveBlock threads):
// workgroup w forms the sum of lanes 64 w .. 64 w + 63 of reduce_partials_at's
// order (thread c * 64 + l takes chunk c of lane 64 w + l; the chunk sums
// are added in order, then the wavefront butterfly) and writes it to
// W[i * kWaves + w].  sum_wave_sums adds W[i * kWaves + 0 .. kWaves - 1] in
// order, which is block_sum's last step: the totals have
// reduce_partials_at's bits.  The wavefronts of chunks without a partial
// below G load nothing.
constexpr int kWaveBlock = 64 * kChunks;

template <int NV, int N1>
__device__ __forceinline__ void wave_partial_sums(const double* __restrict__ P1, const double* __restrict__ P2, int G,
                                                  int Gs, double* __restrict__ W)
{
    __shared__ double cs[kChunks][NV][64];
    const double* P[NV];
    partial_rows<NV, N1>(P1, P2, Gs, P);
    const int l = threadIdx.x & 63;
    const int c = threadIdx.x >> 6;  // chunk, uniform per wavefront
    const int lane = 64 * blockIdx.x + l;
    double sum[NV];
    chunk_sum<NV>(P, lane, c, G, sum);
#pragma unroll
    for (int i = 0; i < NV; ++i) cs[c][i][l] = sum[i];
    __syncthreads();
    if (c == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double a = cs[0][i][l];
#pragma unroll
            for (int q = 1; q < kChunks; ++q) a = a + cs[q][i][l];
            const double v = wave_sum(a);
            if (l == 0) W[i * kWaves + blockIdx.x] = v;
        }
    }
}

template <int NV>
__device__ __forceinline__ void sum_wave_sums(const double* __restrict__ W, double (&t)[NV])
{
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = W[i * kWaves];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) a += W[i * kWaves + q];
        t[i] = a;
    }
}

template <int NV, bool ALL = false, int M>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ P, int G, int Gs, double (&tot)[NV],
                                                double (&lds)[M])
{
    reduce_partials_at<NV, NV, ALL>(P, nullptr, G, Gs, tot, lds);
}

// Stage 1: per-thread sums -> one partial per workgroup and value (value
// i < N1 to P1, the others to P2, with the layout of reduce_partials_at).
template <int NV, int N1>
__device__ __forceinline__ void write_partials_at(double (&acc)[NV], double* __restrict__ P1, double* __restrict__ P2,
                                                  int Gs, int slot, double* lds)
{
    block_sum<NV>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double* P = i < N1 ? P1 + (int64_t)i * Gs : P2 + (int64_t)(i - N1) * Gs;
            P[slot] = acc[i];
        }
    }
}

template <int NV>
__device__ __forceinline__ void write_partials(double (&acc)[NV], double* __restrict__ P, int Gs, int slot,
                                               double* lds)
{
    write_partials_at<NV, NV>(acc, P, nullptr, Gs, slot, lds);
}

// Stage 2 by the last workgroup.  After thread 0 has written the
// workgroup's partials (write_partials), it takes a ticket; the workgroup
// that draws the last one (G - 1) returns true and reduces all partials.
// Thread 0's agent-scope fence before its ticket releases its partials to
// every XCD; the fence after the last ticket (and in every thread of that
// workgroup after the barrier) acquires everyone else's.  No workgroup
// waits for another, so the scheme cannot hang.  The last workgroup resets
// the counter, which is therefore 0 whenever no kernel is running.
__device__ __forceinline__ bool take_last_ticket(int* ticket, int G)
{
    __shared__ int is_last;
    if (threadIdx.x == 0) {
        __threadfence();
        const int t = atomicAdd(ticket, 1);
        const int last = t == G - 1;
        if (last) {
            __threadfence();
            atomicExch(ticket, 0);
        }
        is_last = last;
    }
    __syncthreads();
    const bool last = is_last != 0;
    if (last) __threadfence();
    return last;
}

// Workgroup b of G owns the 256-row groups [g0, g1).  The hardware hands
// workgroups to the 8 XCDs round-robin (b mod 8), so consecutive runs are
// given to workgroups of the same XCD: neighbouring rows then share an L2.
__device__ __forceinline__ void chunk_of(int b, int G, int64_t ngroups, int64_t& g0, int64_t& g1)
{
    int c = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
    g0 = (int64_t)c * ngroups / G;
    g1 = (int64_t)(c + 1) * ngroups / G;
}

// The workgroup whose runs chunk_of gives workgroup b in reverse order:
// each XCD then sweeps its rows from the other end, so a kernel that
// follows one in the forward order starts on the rows that kernel touched
// last, still in the last-level cache.  A kernel that takes its runs this
// way writes its partials at the slot of that workgroup, which keeps the
// reductions' order.
__device__ __forceinline__ int reverse_block(int b, int G)
{
    return (G % 8 == 0) ? b % 8 + 8 * (G / 8 - 1 - b / 8) : G - 1 - b;
}

// Products of one SELL-64 row (entries summed in stored column order; zero
// slots add nothing).  The slots are consumed in fixed-size pieces: K
// values, K columns and K gathered entries are loaded before the first of
// the K multiply-adds, so a piece costs one memory round trip.  Full pieces
// of kChunk slots come first, then one piece of the remaining 1..7 slots,
// selected by a switch on the (wavefront-uniform) slot count, so that no
// load sits behind a per-slot branch.  Offset-aligned and packed slices take
// separate code (one uniform branch per slice): an aligned piece issues the
// scalar loads of its K column offsets together and waits once, where a
// per-slot test had made every slot wait for its own offset (measured on
// MI355X: a 27-point product 1.5x slower).
constexpr int kChunk = 8;

// Column of slot j: offset-aligned (off != nullptr, clamped into
// [first, last] so that zero slots of boundary rows read a valid entry: the
// whole matrix, or the owning system's rows in a block-diagonal batch, so
// that no system reads another's vectors) or packed (explicit).  A zero slot
// still multiplies 0 by the entry it reads: a non-finite vector entry at
// such a column makes the row's result NaN where a CSR product, which has no
// such slot, would stay finite.
struct SlotCols {
    const int32_t* off;
    const int32_t* col;
    int row, first, last;
    int stride;  // elements between consecutive slots of a row
};

// K slots starting at j0; G(c) returns the gathered entry (double or
// double2) at column c, F(acc, a, g) accumulates.
template <int K, bool ALIGNED, class T, bool NT, class Gather, class Acc>
__device__ __forceinline__ void slot_piece(const double* __restrict__ v, const SlotCols& cols, int j0, Gather&& gather,
                                           Acc&& acc)
{
    int c[K];
    if constexpr (ALIGNED) {
        int o[K];
#pragma unroll
        for (int u = 0; u < K; ++u) o[u] = cols.off[j0 + u];  // uniform: scalar loads
#pragma unroll
        for (int u = 0; u < K; ++u) c[u] = min(max(cols.row + o[u], cols.first), cols.last);
    } else {
#pragma unroll
        for (int u = 0; u < K; ++u) c[u] = cols.col[(int64_t)(j0 + u) * cols.stride];
    }
    double a[K];
    T g[K];
#pragma unroll
    for (int u = 0; u < K; ++u) {
        if constexpr (NT)
            a[u] = __builtin_nontemporal_load(v + (int64_t)(j0 + u) * cols.stride);
        else
            a[u] = v[(int64_t)(j0 + u) * cols.stride];
        g[u] = gather(c[u]);
    }
#pragma unroll
    for (int u = 0; u < K; ++u) acc(a[u], g[u]);
}

// The last piece of a row, 1 .. N slots (one uniform branch per size).
template <int N, bool ALIGNED, class T, bool NT, class Gather, class Acc>
__device__ __forceinline__ void slot_rest(int rem, const double* __restrict__ v, const SlotCols& cols, int j0,
                                          Gather&& gather, Acc&& acc)
{
    if constexpr (N >= 1) {
        if (rem == N)
            slot_piece<N, ALIGNED, T, NT>(v, cols, j0, gather, acc);
        else
            slot_rest<N - 1, ALIGNED, T, NT>(rem, v, cols, j0, gather, acc);
    }
}

// Slots of offset-aligned slices per piece (their offsets are scalar loads).
// Measured on MI355X: pieces of 9 take the 27-point product (27 = 3 x 9) from
// 184.4 to 181.2 us against pieces of 8; 14 and 27 were slower (189, 200).
constexpr int kAlignedChunk = 9;

template <bool ALIGNED, class T, bool NT, class Gather, class Acc>
__device__ __forceinline__ void slot_loop_of(const double* __restrict__ v, const SlotCols& cols, int width,
                                             Gather&& gather, Acc&& acc)
{
    constexpr int K = ALIGNED ? kAlignedChunk : kChunk;
    int j0 = 0;
    for (; j0 + K <= width; j0 += K) slot_piece<K, ALIGNED, T, NT>(v, cols, j0, gather, acc);
    slot_rest<K - 1, ALIGNED, T, NT>(width - j0, v, cols, j0, gather, acc);
}

// stream: load the values nontemporally (offset-aligned slices only; a
// packed slice's extra branch would push the pipelined product into spills).
template <class T, class Gather, class Acc>
__device__ __forceinline__ void slot_loop(const double* __restrict__ v, const SlotCols& cols, int width, bool stream,
                                          Gather&& gather, Acc&& acc)
{
    if (cols.off) {
        if (stream)
            slot_loop_of<true, T, true>(v, cols, width, gather, acc);
        else
            slot_loop_of<true, T, false>(v, cols, width, gather, acc);
    } else {
        slot_loop_of<false, T, false>(v, cols, width, gather, acc);
    }
}

__device__ __forceinline__ SlotCols slot_cols(const SellView& A, int64_t slice, int lane, int64_t row64,
                                              int64_t& base, int& width, int first, int last)
{
    base = A.slice_ptr[slice];
    const int32_t shape = A.slice_shape[slice];
    width = shape_width(shape);
    const int meta = A.slice_meta[slice];
    SlotCols c;
    c.off = meta >= 0 ? A.soff + meta : nullptr;
    c.col = A.col + base + lane;
    c.row = (int)row64;
    c.first = first;
    c.last = last;
    c.stride = shape_stride(shape);
    return c;
}

template <int NX>
__device__ __forceinline__ void sell_row(const SellView& A, int64_t slice, int lane, int64_t row64,
                                         const double* __restrict__ x0, const double* __restrict__ x1, double& y0,
                                         double& y1, int first, int last)
{
    int64_t base;
    int width;
    const SlotCols cols = slot_cols(A, slice, lane, row64, base, width, first, last);
    const double* __restrict__ v = A.val + base + lane;
    double a0 = 0.0, a1 = 0.0;
    if (NX == 1) {
        slot_loop<double>(v, cols, width, slice >= A.stream_from, [&](int c) { return x0[c]; },
                          [&](double a, double g) { a0 = fma(a, g, a0); });
    } else {
        slot_loop<double2>(v, cols, width, slice >= A.stream_from, [&](int c) { return make_double2(x0[c], x1[c]); },
                           [&](double a, double2 g) {
                               a0 = fma(a, g.x, a0);
                               a1 = fma(a, g.y, a1);
                           });
    }
    y0 = a0;
    y1 = a1;
}

// A row of the whole matrix: zero slots clamped into [0, n).
template <int NX>
__device__ __forceinline__ void sell_row(const SellView& A, int64_t slice, int lane, int64_t row64,
                                         const double* __restrict__ x0, const double* __restrict__ x1, double& y0,
                                         double& y1)
{
    sell_row<NX>(A, slice, lane, row64, x0, x1, y0, y1, 0, (int)A.n - 1);
}

// Both products of one SELL-64 row with a block vector of pairs:
// (y0, y1) = sum_j a_ij (xy_j.x, xy_j.y), entries in stored column order.
__device__ __forceinline__ void sell_row_pair(const SellView& A, int64_t slice, int lane, int64_t row64,
                                              const double2* __restrict__ xy, double& y0, double& y1)
{
    int64_t base;
    int width;
    const SlotCols cols = slot_cols(A, slice, lane, row64, base, width, 0, (int)A.n - 1);
    const double* __restrict__ v = A.val + base + lane;
    double a0 = 0.0, a1 = 0.0;
    slot_loop<double2>(v, cols, width, slice >= A.stream_from, [&](int c) { return xy[c]; },
                       [&](double a, double2 g) {
                           a0 = fma(a, g.x, a0);
                           a1 = fma(a, g.y, a1);
                       });
    y0 = a0;
    y1 = a1;
}

// Calls f(row, y0, y1) for every row of 256-row group g, where y = A x for
// one or two vectors.  SELL-64: one row per thread.
template <int NX, class F>
__device__ __forceinline__ void sell_group(const SellView& A, int64_t g, const double* __restrict__ x0,
                                           const double* __restrict__ x1, F&& f)
{
    const int w = uniform(threadIdx.x >> 6);
    const int64_t slice = g * kWaves + w;
    if (slice >= A.nslices) return;
    const int lane = threadIdx.x & 63;
    double y0, y1;
    const int64_t row = slice * kSlice + lane;
    sell_row<NX>(A, slice, lane, row, x0, x1, y0, y1);
    if (row < A.n) f(row, y0, y1);
}

// Vector CSR with L lanes per row: the 256 rows of group g are done in L
// passes of 256/L rows; lane 0 of each L-lane team receives the row sums.
template <int L, int NX, class F>
__device__ __forceinline__ void csr_group(const CsrView& A, int64_t g, const double* __restrict__ x0,
                                          const double* __restrict__ x1, F&& f)
{
    const int sub = threadIdx.x % L;
    const int team = threadIdx.x / L;
    for (int q = 0; q < L; ++q) {
        const int64_t row = g * kGroupRows + (int64_t)q * (kBlock / L) + team;
        double a0 = 0.0, a1 = 0.0;
        if (row < A.n) {
            const int32_t e1 = A.row_ptr[row + 1];
            for (int32_t e = A.row_ptr[row] + sub; e < e1; e += L) {
                const double ve = A.val[e];
                const int ce = A.col[e];
                a0 = fma(ve, x0[ce], a0);
                if (NX == 2) a1 = fma(ve, x1[ce], a1);
            }
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off, 64);
            if (NX == 2) a1 += __shfl_xor(a1, off, 64);
        }
        if (sub == 0 && row < A.n) f(row, a0, a1);
    }
}

// Vector-CSR product with a block vector of pairs.
template <int L, class F>
__device__ __forceinline__ void csr_group_pair(const CsrView& A, int64_t g, const double2* __restrict__ xy, F&& f)
{
    const int sub = threadIdx.x % L;
    const int team = threadIdx.x / L;
    for (int q = 0; q < L; ++q) {
        const int64_t row = g * kGroupRows + (int64_t)q * (kBlock / L) + team;
        double a0 = 0.0, a1 = 0.0;
        if (row < A.n) {
            const int32_t e1 = A.row_ptr[row + 1];
            for (int32_t e = A.row_ptr[row] + sub; e < e1; e += L) {
                const double ve = A.val[e];
                const double2 xe = xy[A.col[e]];
                a0 = fma(ve, xe.x, a0);
                a1 = fma(ve, xe.y, a1);
            }
        }
#pragma unroll
        for (int off = L / 2; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off, 64);
            a1 += __shfl_xor(a1, off, 64);
        }
        if (sub == 0 && row < A.n) f(row, a0, a1);
    }
}

template <int LANES, class F>
__device__ __forceinline__ void rows_of_group_pair(const SellView& S, const CsrView& C, int64_t g,
                                                   const double2* __restrict__ xy, F&& f)
{
    if constexpr (LANES == 1) {
        const int w = uniform(threadIdx.x >> 6);
        const int64_t slice = g * kWaves + w;
        if (slice >= S.nslices) return;
        const int lane = threadIdx.x & 63;
        const int64_t row = slice * kSlice + lane;
        double y0, y1;
        sell_row_pair(S, slice, lane, row, xy, y0, y1);
        if (row < S.n) f(row, y0, y1);
    } else {
        csr_group_pair<LANES>(C, g, xy, f);
    }
}

// Dispatch on the storage format (LANES == 1: SELL-64, else vector CSR).
template <int LANES, int NX, class F>
__device__ __forceinline__ void rows_of_group(const SellView& S, const CsrView& C, int64_t g,
                                              const double* __restrict__ x0, const double* __restrict__ x1, F&& f)
{
    if constexpr (LANES == 1)
        sell_group<NX>(S, g, x0, x1, f);
    else
        csr_group<LANES, NX>(C, g, x0, x1, f);
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// Field-by-field copies of the solver state between memory and registers
// (a whole-struct copy can leave part of the struct in a per-thread memory
// array instead of registers).
__device__ __forceinline__ State load_state(const State* __restrict__ p)
{
    State s;
    s.alpha = p->alpha;
    s.beta = p->beta;
    s.nu = p->nu;
    s.mu = p->mu;
    s.sigma = p->sigma;
    s.gamma = p->gamma;
    s.rr = p->rr;
    s.nup = p->nup;
    s.bnorm = p->bnorm;
    s.tol = p->tol;
    s.relres_true = p->relres_true;
    s.k = p->k;
    s.done = p->done;
    s.status = p->status;
    s.last = p->last;
    s.maxit = p->maxit;
    s.zero_x = p->zero_x;
    s.spare0 = s.spare1 = 0;
    s.spare2 = 0.0;
    return s;
}

__device__ __forceinline__ void store_state(State* __restrict__ p, const State& s)
{
    p->alpha = s.alpha;
    p->beta = s.beta;
    p->nu = s.nu;
    p->mu = s.mu;
    p->sigma = s.sigma;
    p->gamma = s.gamma;
    p->rr = s.rr;
    p->nup = s.nup;
    p->bnorm = s.bnorm;
    p->tol = s.tol;
    p->relres_true = s.relres_true;
    p->k = s.k;
    p->done = s.done;
    p->status = s.status;
    p->last = s.last;
    p->maxit = s.maxit;
    p->zero_x = s.zero_x;
}

// The scalar step after the reduction of iteration k of a one-reduction
// variant (PR, M, pipe-PR, pipe-M): record ||r_k||, test convergence and
// breakdown, then form alpha_k, nu'_{k+1} and beta_{k+1} (Alg. 2 / Alg. 3,
// eq. nuk_simplified; Meurant: nu' = -nu + alpha^2 gamma).  form =
// kFormNoRecompute is the ablation of Section 2 that keeps the predicted
// nu'_k as nu_k (eq. nuk_norecomp; nu'_0 := nu_0), so the recomputed inner
// product serves only as ||r_k||^2 when M = I.  form = kFormUnsimplified
// predicts with the four terms of eq. nuk, delta = <s~_k, r_k> (the caller
// passes sigma when M = I, where the two sums are the same); the middle
// terms are grouped as alpha (sigma + delta), which with delta = sigma
// rounds exactly like 2 alpha sigma.
__device__ inline void step_one_reduction(State& st, const double (&t)[5], bool pre, int form, double* hist,
                                          bool writer, double delta = 0.0)
{
    const double mu = t[0], sigma = t[1], gamma = t[2];
    const double nu = (form == kFormNoRecompute && st.k >= 0) ? st.nup : t[3];
    const double rr = pre ? t[4] : t[3];
    const int k = st.k + 1;
    const double rnorm = sqrt(rr > 0.0 ? rr : 0.0);
    if (writer) hist[k] = rnorm / st.bnorm;
    st.k = k;
    st.nu = nu;
    st.mu = mu;
    st.sigma = sigma;
    st.gamma = gamma;
    st.rr = rr;
    if (finite(rr) && rnorm <= st.tol * st.bnorm) {
        st.done = 1;
        st.status = kOK;
        return;
    }
    if (st.last || !finite(nu) || !finite(mu) || !finite(rr) || !(nu > 0.0) || !(mu > 0.0)) {
        st.done = 1;
        st.status = kBreakdown;
        return;
    }
    if (k == st.maxit) {
        st.done = 1;
        st.status = kNotConverged;
        return;
    }
    const double alpha = nu / mu;
    const double nup = form == kFormMeurant        ? -nu + alpha * alpha * gamma
                       : form == kFormUnsimplified ? nu - alpha * (sigma + delta) + alpha * alpha * gamma
                                                   : nu - 2.0 * alpha * sigma + alpha * alpha * gamma;
    st.alpha = alpha;
    st.nup = nup;
    if (!finite(nup) || !(nup > 0.0)) {
        st.last = 1;  // the next iteration's x and r updates are still taken
        st.beta = 0.0;
    } else {
        st.beta = nup / nu;
    }
}

// GV-CG (Appendix D) after the reduction of iteration k >= 1 (nu_k, eta_k
// and, with a preconditioner, <r_k, r_k>): beta_k = nu_k / nu_{k-1},
// mu_k = eta_k - (beta_k / alpha_{k-1}) nu_k, then the tests and
// alpha_k = nu_k / mu_k.
__device__ inline void step_gv(State& st, const double (&t)[3], bool pre, double* hist, bool writer)
{
    const double nu = t[0], eta = t[1];
    const double rr = pre ? t[2] : nu;
    const int k = st.k + 1;
    const double rnorm = sqrt(rr > 0.0 ? rr : 0.0);
    if (writer) hist[k] = rnorm / st.bnorm;
    const double beta = nu / st.nu;
    const double mu = eta - (beta / st.alpha) * nu;
    st.k = k;
    st.rr = rr;
    st.beta = beta;
    st.nu = nu;
    st.mu = mu;
    if (finite(rr) && rnorm <= st.tol * st.bnorm) {
        st.done = 1;
        st.status = kOK;
        return;
    }
    if (!finite(nu) || !finite(mu) || !finite(rr) || !(nu > 0.0) || !(mu > 0.0)) {
        st.done = 1;
        st.status = kBreakdown;
        return;
    }
    if (k == st.maxit) {
        st.done = 1;
        st.status = kNotConverged;
        return;
    }
    st.alpha = nu / mu;
}

// GV-CG at k = 0 (initialize of Appendix D: nu_0, mu_0 and <r_0, r_0> in
// the one-reduction layout t[3], t[0], t[4]): the tests, alpha_0, and
// beta := 0 so that the first direction update leaves p_0, s_0, s~_0, u_0
// as initialised.
__device__ inline void step_gv_first(State& st, const double (&t)[5], bool pre, double* hist, bool writer)
{
    const double mu = t[0], nu = t[3];
    const double rr = pre ? t[4] : nu;
    const double rnorm = sqrt(rr > 0.0 ? rr : 0.0);
    if (writer) hist[0] = rnorm / st.bnorm;
    st.k = 0;
    st.rr = rr;
    st.nu = nu;
    st.mu = mu;
    st.beta = 0.0;
    if (finite(rr) && rnorm <= st.tol * st.bnorm) {
        st.done = 1;
        st.status = kOK;
        return;
    }
    if (!finite(nu) || !finite(mu) || !finite(rr) || !(nu > 0.0) || !(mu > 0.0)) {
        st.done = 1;
        st.status = kBreakdown;
        return;
    }
    if (st.maxit == 0) {
        st.done = 1;
        st.status = kNotConverged;
        return;
    }
    st.alpha = nu / mu;
}

// HS-CG after the reduction of nu_k (Alg. 1): record ||r_k||, test, beta_k.
__device__ inline void step_hs_nu(State& st, double nu, double rr, double* hist, bool writer)
{
    const int k = st.k + 1;
    const double rnorm = sqrt(rr > 0.0 ? rr : 0.0);
    if (writer) hist[k] = rnorm / st.bnorm;
    st.k = k;
    st.rr = rr;
    if (finite(rr) && rnorm <= st.tol * st.bnorm) {
        st.done = 1;
        st.status = kOK;
        st.nu = nu;
        return;
    }
    if (!finite(nu) || !finite(rr) || !(nu > 0.0)) {
        st.done = 1;
        st.status = kBreakdown;
        st.nu = nu;
        return;
    }
    if (k == st.maxit) {
        st.done = 1;
        st.status = kNotConverged;
        st.nu = nu;
        return;
    }
    if (k > 0) st.beta = nu / st.nu;  // beta_k = nu_k / nu_{k-1}
    st.nu = nu;
}

// HS-CG after the reduction of mu_k: alpha_k = nu_k / mu_k.
__device__ inline void step_hs_mu(State& st, double mu)
{
    st.mu = mu;
    if (!finite(mu) || !(mu > 0.0)) {
        st.done = 1;
        st.status = kBreakdown;
        return;
    }
    st.alpha = st.nu / mu;
}

}  // namespace prcg
