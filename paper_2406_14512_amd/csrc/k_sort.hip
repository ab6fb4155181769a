// Stable sort of each species by cell (key = i*nth + j), with the removal
// of particles in the pure force-free domain folded into the key pass.
//
// 1. key pass: one thread per slot; dead slots and particles in kill cells
//    get the dead key (larger than every live key, so they sort last and
//    are dropped), live ones their cell.  Live particles lie inside the
//    absorbing radius, so the dead key is the first cell of the row past
//    it, which keeps the key within 24 bits on a 4096^2 grid (three 8-bit
//    radix passes instead of four).
// 2. rocPRIM LSD radix sort of (key, slot) pairs over the key's bit range:
//    LSD radix sort is stable, so equal keys keep their slot order.
// 3. the live count is the position of the first dead key in the sorted
//    keys (binary search), so no pass of the sort contends on a counter.
// 4. gather pass: the SoA state is permuted into the second buffer.
//
// Between two sorts most particles stay in their cell (a step moves a
// particle by a fraction of a cell), so after the first sort the array is
// re-sorted incrementally (sort_species_incremental):
//   * a particle is a "stayer" if its key equals the key its slot had at the
//     last sort, else a "mover" (dead slots and killed particles drop out);
//     stayers are already in (key, slot) order;
//   * a block scan gives SB[q] = stayers before slot q and compacts the
//     movers (key, slot) in slot order; only the movers are radix sorted;
//   * every particle's place in the stable order by (key, slot) follows
//     from counts: a stayer at q with key k goes to
//       SB[q] + (movers with key < k) + (movers with key k and slot < q),
//     the mover of rank j (key k, slot q) goes to
//       j + SB[clamp(q, OFF[k], OFF[k+1])],
//     with OFF the cell offsets of the last sort (stayers with key < k sit
//     before OFF[k], those with key k inside [OFF[k], OFF[k+1]));
//   * one scatter pass writes the state, the sorted keys and (from the same
//     counts) the new cell offsets, which the next sort compares against.
// The result is the same stable order as a full sort of the keys.
#include <algorithm>
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "device_common.h"

namespace ffpic {

constexpr int kSortBlock = 1024;          // slots per classify / compact block

#define HCHK_SORT(x)                                                                    \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) throw std::runtime_error(hipGetErrorString(e_));          \
    } while (0)

__global__ void k_key64(int nub, const int32_t *__restrict__ nslots, int nr, int nth, double rmin,
                        double dlog, double dth, const double *__restrict__ rn,
                        const double *__restrict__ thn, const uint8_t *__restrict__ kill,
                        uint32_t dead, double *__restrict__ R, const double *__restrict__ TH,
                        uint32_t *__restrict__ keys, uint32_t *__restrict__ vals,
                        unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t key = dead;
    bool killed = false;
    if (q < nslots[0]) {
        double r = R[q];
        if (r > 0.0) {
            int i, j;
            double a, b;
            locate64(nr, nth, rmin, dlog, dth, rn, thn, r, TH[q], i, j, a, b);
            if (kill[(size_t)i * nth + j]) {
                killed = true;
                R[q] = -1.0;
            } else {
                key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
            }
        }
    }
    keys[q] = key;
    if (vals) vals[q] = (uint32_t)q;
    count_wave(&removed[1], killed);
}

__global__ void k_key32(int nub, const int32_t *__restrict__ nslots, int nth,
                        const uint8_t *__restrict__ kill, uint32_t dead,
                        int32_t *__restrict__ CELL, uint32_t *__restrict__ keys,
                        uint32_t *__restrict__ vals, unsigned long long *__restrict__ removed) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t key = dead;
    bool killed = false;
    if (q < nslots[0]) {
        int c = CELL[q];
        if (c >= 0) {
            int i = c >> 16, j = c & 0xffff;
            if (kill[(size_t)i * nth + j]) {
                killed = true;
                CELL[q] = -1;
            } else {
                key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
            }
        }
    }
    keys[q] = key;
    if (vals) vals[q] = (uint32_t)q;
    count_wave(&removed[1], killed);
}

// number of live keys = index of the first dead key in the sorted keys
__global__ void k_count_sorted(int nub, const uint32_t *__restrict__ keys, uint32_t dead,
                               int32_t *__restrict__ nalive, int32_t *__restrict__ nslots,
                               int32_t *__restrict__ nsorted) {
    int lo = 0, hi = nub;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (keys[mid] < dead) lo = mid + 1; else hi = mid;
    }
    nalive[0] = lo;
    if (nslots) nslots[0] = lo;
    if (nsorted) nsorted[0] = lo;
}

// live count of unsorted keys: block reduction, one atomic per block
__global__ void __launch_bounds__(256) k_count_live(int nub, const uint32_t *__restrict__ keys,
                                                    uint32_t dead, int32_t *__restrict__ nalive) {
    __shared__ int part[4];
    int c = 0;
    for (int q = blockIdx.x * 256 + threadIdx.x; q < nub; q += gridDim.x * 256) c += keys[q] < dead;
    for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(nalive, part[0] + part[1] + part[2] + part[3]);
}

// permutes all state arrays of a species in one pass over the permutation
template <typename T, int NA>
struct PtrSet {
    const T *src[NA];
    T *dst[NA];
};

template <typename T, int NA>
__global__ void k_gather_set(int nub, const int32_t *__restrict__ nalive,
                             const uint32_t *__restrict__ perm, PtrSet<T, NA> P) {
    const int n = min(nub, nalive[0]);
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const uint32_t s = perm[q];
        T v[NA];
#pragma unroll
        for (int a = 0; a < NA; a++) v[a] = P.src[a][s];
#pragma unroll
        for (int a = 0; a < NA; a++) P.dst[a][q] = v[a];
    }
}

__global__ void k_zero_i32(int32_t *p, int n) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0;
}

void zero_counters(ffpic_ctx *c, int32_t *p, int n) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 63) / 64), dim3(64), 0, c->stream, p, n);
}

// first key past every live one (see the header comment)
static uint32_t dead_key(const ffpic_ctx *c) {
    double xa = std::log(c->d.r_abs / c->d.rmin) / c->dlog;
    int64_t iabs = (int64_t)std::floor(xa);
    int64_t k = (iabs + 1) * (int64_t)c->nth;
    int64_t all = (int64_t)c->nr * c->nth;
    return (uint32_t)(iabs + 1 < c->nr ? k : all);
}

int sort_key_bits(const ffpic_ctx *c) {
    uint64_t dead = dead_key(c);
    int bits = 1;
    while ((1ull << bits) <= dead) bits++;
    return bits;
}

size_t scan_temp_bytes(int64_t nblk) {
    size_t bytes = 0;
    if (nblk <= 0) return 0;
    hipError_t e = rocprim::exclusive_scan((void *)nullptr, bytes, (uint32_t *)nullptr,
                                           (uint32_t *)nullptr, 0u, (size_t)nblk,
                                           rocprim::plus<uint32_t>());
    if (e != hipSuccess) throw std::runtime_error("rocprim scan size query failed");
    return bytes;
}

int sort_block_slots() { return kSortBlock; }

// temporary storage for sorting any number of pairs up to cap: rocPRIM
// switches algorithm with the size (merge sort below about 2^20 items), so
// the largest requirement over the switch points is taken
size_t sort_temp_bytes(int64_t cap, int bits) {
    if (cap <= 0) return 0;
    size_t most = 0;
    const int64_t sizes[] = {cap, std::min<int64_t>(cap, (1 << 20) - 1),
                             std::min<int64_t>(cap, (1 << 20) + 1)};
    for (int64_t n : sizes) {
        size_t bytes = 0;
        hipError_t e = rocprim::radix_sort_pairs((void *)nullptr, bytes, (uint32_t *)nullptr,
                                                 (uint32_t *)nullptr, (uint32_t *)nullptr,
                                                 (uint32_t *)nullptr, (unsigned int)n, 0, bits);
        if (e != hipSuccess) throw std::runtime_error("rocprim temp size query failed");
        most = std::max(most, bytes);
    }
    return most;
}

static void key_pass(ffpic_ctx *c, int s, uint32_t dead, bool with_vals = true) {
    ffpic::Species &S = c->sp[s];
    int nub = (int)S.nub;
    int nb = (nub + 255) / 256;
    if (c->fp64) {
        hipLaunchKernelGGL(k_key64, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nr,
                           c->nth, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN], c->dtab64[T_THN],
                           c->kill, dead, (double *)S.cur[0], (const double *)S.cur[1],
                           c->keys[0], with_vals ? c->vals[0] : nullptr, c->removed + 4 * s);
    } else {
        hipLaunchKernelGGL(k_key32, dim3(nb), dim3(256), 0, c->stream, nub, c->nslots + s, c->nth,
                           c->kill, dead, (int32_t *)S.cur[0], c->keys[0],
                           with_vals ? c->vals[0] : nullptr, c->removed + 4 * s);
    }
    FFPIC_LAUNCH_CHECK();
}

// removal of particles in force-free cells without reordering
void kill_species(ffpic_ctx *c, int s) {
    if (c->sp[s].nub == 0) return;
    key_pass(c, s, dead_key(c));
}

// cell offsets from the current (sorted) order: off[k] = first slot whose
// key is >= k, found by binary search over the live slots
__global__ void k_offsets(int nalive_host, const uint32_t *__restrict__ keys, int nkeys,
                          int32_t *__restrict__ off) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int lo = 0, hi = nalive_host;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((int)keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    off[k] = lo;
}

void sort_offsets(ffpic_ctx *c, int s, int32_t *dev_off) {
    // keys of the current order (no removal): all-zero kill flags
    ffpic::Species &S = c->sp[s];
    int nkeys = c->nr * c->nth;
    int nal = 0;
    if (S.nub > 0) {
        uint8_t *nok = nullptr;
        size_t ncell = (size_t)c->nr * c->nth;
        if (hipMalloc(&nok, ncell) != hipSuccess) throw std::runtime_error("hipMalloc failed");
        (void)hipMemsetAsync(nok, 0, ncell, c->stream);
        uint8_t *saved = c->kill;
        c->kill = nok;
        uint32_t dead = dead_key(c);
        key_pass(c, s, dead);
        c->kill = saved;
        zero_counters(c, c->nalive + s, 1);
        hipLaunchKernelGGL(k_count_live, dim3(256), dim3(256), 0, c->stream, (int)S.nub,
                           c->keys[0], dead, c->nalive + s);
        (void)hipMemcpyAsync(&nal, c->nalive + s, sizeof(int), hipMemcpyDeviceToHost, c->stream);
        (void)hipStreamSynchronize(c->stream);
        (void)hipFree(nok);
    }
    hipLaunchKernelGGL(k_offsets, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream, nal,
                       c->keys[0], nkeys, dev_off);
    FFPIC_LAUNCH_CHECK();
}


// ---------------------------------------------------------------------------
// incremental re-sort


// stayer / mover class of a slot from its new key and the key it had at the
// last sort (kold is sorted, so stayers are in order)
__device__ __forceinline__ int slot_class(uint32_t key, uint32_t dead, int q, int nold,
                                          const uint32_t *__restrict__ kold) {
    if (key >= dead) return 0;                          // dropped
    return (q < nold && kold[q] == key) ? 1 : 2;        // 1 stayer, 2 mover
}

// key pass fused with the stayer / mover counts of each block of
// kSortBlock slots (incremental sort); same keys and removals as k_key32 /
// k_key64
__device__ __forceinline__ void block_counts(uint32_t st, uint32_t mv, uint32_t *bst,
                                             uint32_t *bmv) {
    __shared__ uint32_t part[2][4];
    const int tid = threadIdx.x, w = tid >> 6;
    if ((tid & 63) == 0) { part[0][w] = st; part[1][w] = mv; }
    __syncthreads();
    if (tid == 0) {
        bst[blockIdx.x] = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        bmv[blockIdx.x] = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    }
}

// FP32 key pass of the incremental sort: kill, then the class of every slot
// (0 dropped, 1 stayer, 2 mover) as one byte, with the block counts.  The
// later passes take the key of a slot from its cell, so no key array is
// written.  The loads of the block's four slots per thread are issued first.
__global__ void __launch_bounds__(256) k_keyclass32(int nub, const int32_t *__restrict__ nslots,
                                                    int nth, const uint8_t *__restrict__ kill,
                                                    uint32_t dead, int32_t *__restrict__ CELL,
                                                    uint8_t *__restrict__ cls,
                                                    unsigned long long *__restrict__ removed,
                                                    const int32_t *__restrict__ nsorted,
                                                    const uint32_t *__restrict__ kold,
                                                    uint32_t *__restrict__ bst,
                                                    uint32_t *__restrict__ bmv) {
    constexpr int K = kSortBlock / 256;
    const int ns = nslots[0], no = nsorted[0];
    int cell[K];
    uint32_t ko[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + threadIdx.x;
        cell[k] = q < ns ? CELL[q] : -1;
        ko[k] = q < no ? kold[q] : dead;
    }
    uint32_t st = 0, mv = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + threadIdx.x;
        const int c = cell[k];
        bool killed = false;
        int cl = 0;
        if (c >= 0) {
            const int i = c >> 16, j = c & 0xffff;
            if (kill[(size_t)i * nth + j]) {
                killed = true;
                CELL[q] = -1;
            } else {
                const uint32_t key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
                cl = key >= dead ? 0 : (key == ko[k] ? 1 : 2);
            }
        }
        if (q < nub) cls[q] = (uint8_t)cl;
        count_wave(&removed[1], killed);
        st += __popcll(__ballot(cl == 1));
        mv += __popcll(__ballot(cl == 2));
    }
    block_counts(st, mv, bst, bmv);
}

__global__ void __launch_bounds__(256) k_keyclass64(
    int nub, const int32_t *__restrict__ nslots, int nr, int nth, double rmin, double dlog,
    double dth, const double *__restrict__ rn, const double *__restrict__ thn,
    const uint8_t *__restrict__ kill, uint32_t dead, double *__restrict__ R,
    const double *__restrict__ TH, uint32_t *__restrict__ keys,
    unsigned long long *__restrict__ removed, const int32_t *__restrict__ nsorted,
    const uint32_t *__restrict__ kold, uint32_t *__restrict__ bst, uint32_t *__restrict__ bmv) {
    const int ns = nslots[0], no = nsorted[0];
    uint32_t st = 0, mv = 0;
    for (int k = 0; k < kSortBlock / 256; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + threadIdx.x;
        uint32_t key = dead;
        bool killed = false;
        if (q < ns) {
            const double r = R[q];
            if (r > 0.0) {
                int i, j;
                double a, b;
                locate64(nr, nth, rmin, dlog, dth, rn, thn, r, TH[q], i, j, a, b);
                if (kill[(size_t)i * nth + j]) {
                    killed = true;
                    R[q] = -1.0;
                } else {
                    key = (uint32_t)i * (uint32_t)nth + (uint32_t)j;
                }
            }
        }
        if (q < nub) keys[q] = key;
        count_wave(&removed[1], killed);
        const int cl = q < nub ? slot_class(key, dead, q, no, kold) : 0;
        st += __popcll(__ballot(cl == 1));
        mv += __popcll(__ballot(cl == 2));
    }
    block_counts(st, mv, bst, bmv);
}

// SB[q] for every slot (stayers before q), the movers compacted in slot
// order, and the totals (SB[nub] = stayers, tot[0] = stayers, tot[1] =
// movers) from the exclusive block scans
__global__ void __launch_bounds__(256) k_class_compact(
    int nub, int nblk, const uint32_t *__restrict__ keys, uint32_t dead,
    const int32_t *__restrict__ nold, const uint32_t *__restrict__ kold,
    const uint32_t *__restrict__ bst, const uint32_t *__restrict__ bmv,
    const uint32_t *__restrict__ cst, const uint32_t *__restrict__ cmv, uint32_t *__restrict__ sb,
    uint32_t *__restrict__ mkey, uint32_t *__restrict__ mval, uint32_t *__restrict__ tot) {
    __shared__ uint32_t part[2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int no = nold[0];
    uint32_t st0 = cst[blockIdx.x], mv0 = cmv[blockIdx.x];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int k = 0; k < kSortBlock / 256; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + tid;
        const uint32_t key = q < nub ? keys[q] : dead;
        const int cl = q < nub ? slot_class(key, dead, q, no, kold) : 0;
        const unsigned long long ms = __ballot(cl == 1), mm = __ballot(cl == 2);
        if (lane == 0) { part[0][w] = __popcll(ms); part[1][w] = __popcll(mm); }
        __syncthreads();
        uint32_t os = st0, om = mv0;
        for (int u = 0; u < w; u++) { os += part[0][u]; om += part[1][u]; }
        os += __popcll(ms & below);
        om += __popcll(mm & below);
        if (q < nub) sb[q] = os;
        if (cl == 2) { mkey[om] = key; mval[om] = (uint32_t)q; }
        st0 += part[0][0] + part[0][1] + part[0][2] + part[0][3];
        mv0 += part[1][0] + part[1][1] + part[1][2] + part[1][3];
        __syncthreads();
    }
    if (blockIdx.x == nblk - 1 && tid == 0) {
        sb[nub] = st0;
        tot[0] = st0;
        tot[1] = mv0;
    }
}

// FP32 variant of the compaction: classes from the byte array, the key of a
// mover from its cell
__global__ void __launch_bounds__(256) k_class_compact32(
    int nub, int nblk, int nth, const uint8_t *__restrict__ cls, const int32_t *__restrict__ CELL,
    const uint32_t *__restrict__ cst, const uint32_t *__restrict__ cmv, uint32_t *__restrict__ sb,
    uint32_t *__restrict__ mkey, uint32_t *__restrict__ mval, uint32_t *__restrict__ tot) {
    constexpr int K = kSortBlock / 256;
    // per-wave counts, double-buffered: a wave writes buffer k & 1 only after
    // the barrier of pass k - 1, which every wave passes after its reads of
    // pass k - 2, so one barrier per pass suffices
    __shared__ uint32_t part[2][2][4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    int cl[K], cc[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + tid;
        cl[k] = q < nub ? (int)cls[q] : 0;
    }
    // the movers' cells are loaded before the passes, off their barriers
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + tid;
        cc[k] = cl[k] == 2 ? CELL[q] : 0;
    }
    uint32_t st0 = cst[blockIdx.x], mv0 = cmv[blockIdx.x];
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int q = blockIdx.x * kSortBlock + k * 256 + tid;
        uint32_t(*pt)[4] = part[k & 1];
        const unsigned long long ms = __ballot(cl[k] == 1), mm = __ballot(cl[k] == 2);
        if (lane == 0) { pt[0][w] = __popcll(ms); pt[1][w] = __popcll(mm); }
        __syncthreads();
        uint32_t os = st0, om = mv0;
        for (int u = 0; u < w; u++) { os += pt[0][u]; om += pt[1][u]; }
        os += __popcll(ms & below);
        om += __popcll(mm & below);
        if (q < nub) sb[q] = os;
        if (cl[k] == 2) {
            const int c = cc[k];
            mkey[om] = (uint32_t)(c >> 16) * (uint32_t)nth + (uint32_t)(c & 0xffff);
            mval[om] = (uint32_t)q;
        }
        st0 += pt[0][0] + pt[0][1] + pt[0][2] + pt[0][3];
        mv0 += pt[1][0] + pt[1][1] + pt[1][2] + pt[1][3];
    }
    if (blockIdx.x == nblk - 1 && tid == 0) {
        sb[nub] = st0;
        tot[0] = st0;
        tot[1] = mv0;
    }
}

// moff[k] = movers with key < k (binary search in the sorted mover keys)
__global__ void k_mover_offsets(const uint32_t *__restrict__ tot, const uint32_t *__restrict__ mkey,
                                int nkeys, int32_t *__restrict__ moff) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int lo = 0, hi = (int)tot[1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)mkey[mid] < k) lo = mid + 1; else hi = mid;
    }
    moff[k] = lo;
}

// mst[k] = moff[k] + (movers of key k from a slot below OFF[k]).  A stayer
// of key k sits in the old range [OFF[k], OFF[k+1]) of its key, and no mover
// of key k does (its key changed, or it was appended after the sort), so
// every stayer of key k has the same movers of its key before it: mst[k].
__global__ void k_mover_start(int nkeys, const int32_t *__restrict__ moff,
                              const int32_t *__restrict__ offold,
                              const uint32_t *__restrict__ mval, int32_t *__restrict__ mst) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int lo = moff[k];
    if (k < nkeys) {
        int hi = moff[k + 1];
        const int q0 = offold[k];
        while (lo < hi) {                 // movers of this key are in slot order
            const int mid = (lo + hi) >> 1;
            if ((int)mval[mid] < q0) lo = mid + 1; else hi = mid;
        }
    }
    mst[k] = lo;
}

// stayers: slot q with key k goes to SB[q] + mst[k]
// One kernel places both classes: the first nbm blocks stride over the
// sorted movers (dispatched first, so their dependent loads overlap the
// streaming copy), the remaining blocks take one slot per thread (stayers).
//   stayer: slot q with key k goes to SB[q] + mst[k];
//   mover:  rank j (key k, slot q) goes to j + SB[clamp(q, OFF[k], OFF[k+1])].
template <typename T, int NA>
__global__ void k_scatter(int nub, int nbm, const uint32_t *__restrict__ keys, uint32_t dead,
                          const int32_t *__restrict__ nold, const uint32_t *__restrict__ kold,
                          const uint32_t *__restrict__ sb, const int32_t *__restrict__ mst,
                          const uint32_t *__restrict__ tot, const uint32_t *__restrict__ mkey,
                          const uint32_t *__restrict__ mval, const int32_t *__restrict__ offold,
                          uint32_t *__restrict__ knew, PtrSet<T, NA> P) {
    if ((int)blockIdx.x < nbm) {
        const int m = (int)tot[1];
        for (int j = (int)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += nbm * blockDim.x) {
            const uint32_t key = mkey[j];
            const int q = (int)mval[j];
            const int lo = offold[key], hi = offold[key + 1];
            const int c = q < lo ? lo : (q > hi ? hi : q);
            const uint32_t d = (uint32_t)j + sb[c];
#pragma unroll
            for (int a = 0; a < NA; a++) P.dst[a][d] = P.src[a][q];
            knew[d] = key;
        }
        return;
    }
    const int q = ((int)blockIdx.x - nbm) * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    // the state is read before the class is known, so its loads overlap the
    // key and offset loads (dead slots are read and dropped)
    T v[NA];
#pragma unroll
    for (int a = 0; a < NA; a++) v[a] = P.src[a][q];
    const uint32_t key = keys[q];
    if (slot_class(key, dead, q, nold[0], kold) != 1) return;
    const uint32_t d = sb[q] + (uint32_t)mst[key];
#pragma unroll
    for (int a = 0; a < NA; a++) P.dst[a][d] = v[a];
    knew[d] = key;
}

// FP32 variant of the scatter: a stayer's class from the byte array and its
// key from its cell (the first state array)
__global__ void k_scatter32(int nub, int nbm, int nth, const uint8_t *__restrict__ cls,
                            const uint32_t *__restrict__ sb, const int32_t *__restrict__ mst,
                            const uint32_t *__restrict__ tot, const uint32_t *__restrict__ mkey,
                            const uint32_t *__restrict__ mval, const int32_t *__restrict__ offold,
                            uint32_t *__restrict__ knew, PtrSet<uint32_t, 6> P) {
    if ((int)blockIdx.x < nbm) {
        const int m = (int)tot[1];
        for (int j = (int)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += nbm * blockDim.x) {
            const uint32_t key = mkey[j];
            const int q = (int)mval[j];
            const int lo = offold[key], hi = offold[key + 1];
            const int c = q < lo ? lo : (q > hi ? hi : q);
            const uint32_t d = (uint32_t)j + sb[c];
#pragma unroll
            for (int a = 0; a < 6; a++) P.dst[a][d] = P.src[a][q];
            knew[d] = key;
        }
        return;
    }
    const int q = ((int)blockIdx.x - nbm) * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t v[6];
#pragma unroll
    for (int a = 0; a < 6; a++) v[a] = P.src[a][q];
    if (cls[q] != 1) return;
    const int cell = (int)v[0];
    const uint32_t key = (uint32_t)(cell >> 16) * (uint32_t)nth + (uint32_t)(cell & 0xffff);
    const uint32_t d = sb[q] + (uint32_t)mst[key];
#pragma unroll
    for (int a = 0; a < 6; a++) P.dst[a][d] = v[a];
    knew[d] = key;
}

// The same placement in two passes, for sorts whose non-stayers fit the
// compact buffer.  The stayer pass reads every slot once (coalesced), places
// the stayers, and copies the state of each mover to the buffer at q - SB[q]
// (the non-stayers before q), so the movers' writes there are coalesced too.
// The mover pass then reads the movers' state from that dense buffer instead
// of from their scattered old slots.
__global__ void k_scatter32_stay(int nub, int nth, const uint8_t *__restrict__ cls,
                                 const uint32_t *__restrict__ sb, const int32_t *__restrict__ mst,
                                 uint32_t *__restrict__ knew, PtrSet<uint32_t, 6> P,
                                 uint32_t *__restrict__ cbuf, int64_t cn) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nub) return;
    uint32_t v[6];
#pragma unroll
    for (int a = 0; a < 6; a++) v[a] = P.src[a][q];
    const int cl = cls[q];
    if (cl == 1) {
        const int cell = (int)v[0];
        const uint32_t key = (uint32_t)(cell >> 16) * (uint32_t)nth + (uint32_t)(cell & 0xffff);
        const uint32_t d = sb[q] + (uint32_t)mst[key];
#pragma unroll
        for (int a = 0; a < 6; a++) P.dst[a][d] = v[a];
        knew[d] = key;
    } else if (cl == 2) {
        const size_t t = (size_t)((uint32_t)q - sb[q]);
#pragma unroll
        for (int a = 0; a < 6; a++) cbuf[(size_t)a * (size_t)cn + t] = v[a];
    }
}

__global__ void k_scatter32_move(int nbm, const uint32_t *__restrict__ tot,
                                 const uint32_t *__restrict__ mkey,
                                 const uint32_t *__restrict__ mval,
                                 const int32_t *__restrict__ offold,
                                 const uint32_t *__restrict__ sb, uint32_t *__restrict__ knew,
                                 PtrSet<uint32_t, 6> P, const uint32_t *__restrict__ cbuf,
                                 int64_t cn) {
    const int m = (int)tot[1];
    for (int j = (int)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += nbm * blockDim.x) {
        const uint32_t key = mkey[j];
        const int q = (int)mval[j];
        const int lo = offold[key], hi = offold[key + 1];
        const int c = q < lo ? lo : (q > hi ? hi : q);
        const uint32_t d = (uint32_t)j + sb[c];
        const size_t t = (size_t)((uint32_t)q - sb[q]);
#pragma unroll
        for (int a = 0; a < 6; a++) P.dst[a][d] = cbuf[(size_t)a * (size_t)cn + t];
        knew[d] = key;
    }
}

// offsets of the new order: stayers with key < k (= SB at the old offset)
// plus movers with key < k; the last entry is the live count
__global__ void k_new_offsets(int nkeys, const int32_t *__restrict__ offold,
                              const uint32_t *__restrict__ sb, const int32_t *__restrict__ moff,
                              int32_t *__restrict__ offnew, int32_t *__restrict__ nalive,
                              int32_t *__restrict__ nslots, int32_t *__restrict__ nsorted) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    const int v = (int)sb[offold[k]] + moff[k];
    offnew[k] = v;
    if (k == nkeys) {
        nalive[0] = v;
        nslots[0] = v;
        nsorted[0] = v;
    }
}

// offsets of a sorted key array (after a full sort): off[k] = first slot
// with key >= k among the live ones
__global__ void k_offsets_dev(const int32_t *__restrict__ nalive, const uint32_t *__restrict__ keys,
                              int nkeys, int32_t *__restrict__ off) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > nkeys) return;
    int lo = 0, hi = nalive[0];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)keys[mid] < k) lo = mid + 1; else hi = mid;
    }
    off[k] = lo;
}

template <typename T, int NA>
static PtrSet<T, NA> state_ptrs(ffpic::Species &S) {
    PtrSet<T, NA> P;
    for (int a = 0; a < NA; a++) {
        P.src[a] = (const T *)S.cur[a];
        P.dst[a] = (T *)S.alt[a];
    }
    return P;
}

// full sort: key pass, radix sort of all (key, slot) pairs, gather; then the
// sorted keys and cell offsets are kept for the next (incremental) sort
static void sort_full(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    int nub = (int)S.nub;
    uint32_t dead = dead_key(c);
    key_pass(c, s, dead);
    size_t bytes = c->sort_tmp_bytes;
    hipError_t e = rocprim::radix_sort_pairs(c->sort_tmp, bytes, c->keys[0], c->keys[1],
                                             c->vals[0], c->vals[1], (unsigned int)nub, 0,
                                             sort_key_bits(c), c->stream);
    if (e != hipSuccess) throw std::runtime_error("rocprim radix sort failed");
    int32_t *nal = c->nalive + s;
    hipLaunchKernelGGL(k_count_sorted, dim3(1), dim3(1), 0, c->stream, nub, c->keys[1], dead, nal,
                       c->nslots + s, c->nsorted + s);
    int nb = std::min((nub + 255) / 256, 65536);
    if (c->fp64) {
        hipLaunchKernelGGL((k_gather_set<uint64_t, 5>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, c->vals[1], (state_ptrs<uint64_t, 5>(S)));
    } else {
        hipLaunchKernelGGL((k_gather_set<uint32_t, 6>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, c->vals[1], (state_ptrs<uint32_t, 6>(S)));
    }
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
    // the sorted keys and their cell offsets, for the next sort
    const int t = c->sort_cur[s];
    HCHK_SORT(hipMemcpyAsync(c->skey[s][t], c->keys[1], (size_t)nub * 4, hipMemcpyDeviceToDevice,
                             c->stream));
    const int nkeys = c->nr * c->nth;
    hipLaunchKernelGGL(k_offsets_dev, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream, nal,
                       c->skey[s][t], nkeys, c->soff[s][t]);
    FFPIC_LAUNCH_CHECK();
    c->sort_valid[s] = true;
}

// incremental sort (see the header comment); requires the keys and offsets
// of the previous sort of this species
static void sort_incremental(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    const int nub = (int)S.nub;
    const uint32_t dead = dead_key(c);
    const int nkeys = c->nr * c->nth;
    const int t = c->sort_cur[s];
    const uint32_t *kold = c->skey[s][t];
    const int32_t *offold = c->soff[s][t];
    const int32_t *nold = c->nsorted + s;  // live count of the last sort
    const int nblk = (nub + kSortBlock - 1) / kSortBlock;
    uint32_t *bst = c->sort_blk, *bmv = bst + nblk, *cst = bmv + nblk, *cmv = cst + nblk;
    if (c->fp64) {
        hipLaunchKernelGGL(k_keyclass64, dim3(nblk), dim3(256), 0, c->stream, nub, c->nslots + s,
                           c->nr, c->nth, c->d.rmin, c->dlog, c->dth, c->dtab64[T_RN],
                           c->dtab64[T_THN], c->kill, dead, (double *)S.cur[0],
                           (const double *)S.cur[1], c->keys[0], c->removed + 4 * s, nold, kold,
                           bst, bmv);
    } else {
        hipLaunchKernelGGL(k_keyclass32, dim3(nblk), dim3(256), 0, c->stream, nub, c->nslots + s,
                           c->nth, c->kill, dead, (int32_t *)S.cur[0], c->sort_cls,
                           c->removed + 4 * s, nold, kold, bst, bmv);
    }
    FFPIC_LAUNCH_CHECK();
    size_t bytes = c->scan_tmp_bytes;
    if (rocprim::exclusive_scan(c->scan_tmp, bytes, bst, cst, 0u, (size_t)nblk,
                                rocprim::plus<uint32_t>(), c->stream) != hipSuccess ||
        rocprim::exclusive_scan(c->scan_tmp, bytes, bmv, cmv, 0u, (size_t)nblk,
                                rocprim::plus<uint32_t>(), c->stream) != hipSuccess)
        throw std::runtime_error("rocprim scan failed");
    uint32_t *mkey = c->keys[1], *mval = c->vals[0];
    if (c->fp64)
        hipLaunchKernelGGL(k_class_compact, dim3(nblk), dim3(256), 0, c->stream, nub, nblk,
                           c->keys[0], dead, nold, kold, bst, bmv, cst, cmv, c->sort_sb, mkey, mval,
                           c->sort_tot);
    else
        hipLaunchKernelGGL(k_class_compact32, dim3(nblk), dim3(256), 0, c->stream, nub, nblk,
                           c->nth, c->sort_cls, (const int32_t *)S.cur[0], cst, cmv, c->sort_sb,
                           mkey, mval, c->sort_tot);
    FFPIC_LAUNCH_CHECK();
    uint32_t tot[2] = {0, 0};
    HCHK_SORT(hipMemcpyAsync(tot, c->sort_tot, sizeof(tot), hipMemcpyDeviceToHost, c->stream));
    HCHK_SORT(hipStreamSynchronize(c->stream));
    const uint32_t m = tot[1];
    uint32_t *mkey2 = c->vals[1], *mval2 = c->sort_aux;
    if (m > 0) {
        size_t sbytes = c->sort_tmp_bytes;
        if (rocprim::radix_sort_pairs(c->sort_tmp, sbytes, mkey, mkey2, mval, mval2, m, 0,
                                      sort_key_bits(c), c->stream) != hipSuccess)
            throw std::runtime_error("rocprim radix sort failed");
    }
    hipLaunchKernelGGL(k_mover_offsets, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream,
                       c->sort_tot, mkey2, nkeys, c->sort_moff);
    hipLaunchKernelGGL(k_mover_start, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream,
                       nkeys, c->sort_moff, offold, mval2, c->sort_mst);
    uint32_t *knew = c->skey[s][1 - t];
    int32_t *offnew = c->soff[s][1 - t];
    const int nbs = (nub + 255) / 256;
    const int nbm = std::max(1, std::min((int)((m + 255) / 256), 4096));
    if (c->fp64) {
        hipLaunchKernelGGL((k_scatter<uint64_t, 5>), dim3(nbs + nbm), dim3(256), 0, c->stream,
                           nub, nbm, c->keys[0], dead, nold, kold, c->sort_sb, c->sort_mst,
                           c->sort_tot, mkey2, mval2, offold, knew, (state_ptrs<uint64_t, 5>(S)));
    } else if (c->sort_cbuf && (int64_t)nub - (int64_t)tot[0] <= c->sort_cbuf_n) {
        const auto P = state_ptrs<uint32_t, 6>(S);
        hipLaunchKernelGGL(k_scatter32_stay, dim3(nbs), dim3(256), 0, c->stream, nub, c->nth,
                           c->sort_cls, c->sort_sb, c->sort_mst, knew, P, c->sort_cbuf,
                           c->sort_cbuf_n);
        hipLaunchKernelGGL(k_scatter32_move, dim3(nbm), dim3(256), 0, c->stream, nbm, c->sort_tot,
                           mkey2, mval2, offold, c->sort_sb, knew, P, c->sort_cbuf,
                           c->sort_cbuf_n);
    } else {
        hipLaunchKernelGGL(k_scatter32, dim3(nbs + nbm), dim3(256), 0, c->stream, nub, nbm,
                           c->nth, c->sort_cls, c->sort_sb, c->sort_mst, c->sort_tot, mkey2,
                           mval2, offold, knew, (state_ptrs<uint32_t, 6>(S)));
    }
    // reads the old live count before replacing it with the new one
    hipLaunchKernelGGL(k_new_offsets, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream,
                       nkeys, offold, c->sort_sb, c->sort_moff, offnew, c->nalive + s,
                       c->nslots + s, c->nsorted + s);
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
    c->sort_cur[s] = 1 - t;
}

void sort_species(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    if (c->sort_valid[s] && c->incremental_sort) sort_incremental(c, s);
    else sort_full(c, s);
}

}  // namespace ffpic
