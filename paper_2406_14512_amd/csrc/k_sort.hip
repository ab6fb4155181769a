// Stable sort of each species by cell (key = i*nth + j), with the removal
// of particles in the pure force-free domain folded into the key pass.  No
// step of it reads anything back to the host: every count lives on the
// device, and every launch is sized by the host bound of the slots, so a
// sort can be captured in a graph.
//
// Full sort (the first sort of a species, or after a load):
//   1. key pass: dead slots and particles in kill cells get the dead key
//      (larger than every live key: the first cell of the row past the
//      absorbing radius, so keys of a 4096^2 grid fit 24 bits), live ones
//      their cell, paired with their slot;
//   2. LSD radix sort of the (key, slot) pairs, 8-bit digits: per tile of
//      4096 pairs a digit histogram, a scan of the histograms of each digit
//      over the tiles, and a stable scatter that ranks equal digits inside
//      a tile in slot order (so equal keys keep their slot order);
//   3. the live count is the position of the first dead key;
//   4. the state is gathered into the second buffer.
//
// Incremental sort (every later sort).  Between two sorts few particles
// change cell, so only those are sorted:
//   * a slot holds a "stayer" if its particle's key equals the key the slot
//     had at the last sort, a "mover" otherwise (dead slots and killed
//     particles drop out); the stayers are already in (key, slot) order.
//     The key a slot had is read off that sort's cell offsets: it is the
//     key whose range [OFF[k], OFF[k+1]) holds the slot;
//   * the classify pass writes one stayer and one mover bit per slot (a
//     64-bit word per 64 slots, from a wave ballot), the counts of both
//     before each word inside its tile of 2048 slots, and the tile's movers
//     (key, slot) compacted inside the tile; two small scans turn the tile
//     counts into exclusive prefixes, so SB(x), the stayers before slot x,
//     and MB(x), the movers before x, are a few loads and a popcount;
//   * the movers are compacted into one array (slot order) and radix
//     sorted as above (stable, so by (key, slot));
//   * each particle's place in the stable order by (key, slot) follows from
//     counts: a stayer at q with key k goes to
//       SB(q) + (movers with key < k) + (movers with key k and slot < q),
//     the mover of rank j (key k, slot q) goes to
//       j + SB(clamp(q, OFF[k], OFF[k+1])),
//     with OFF the cell offsets of the last sort (stayers with key < k sit
//     before OFF[k], those with key k inside [OFF[k], OFF[k+1]), and no
//     mover of key k does);
//   * one pass over the keys gives, per key, the movers-before term of the
//     stayers and the new cell offsets SB(OFF[k]) + (movers with key < k);
//   * the stayer pass reads every slot once and writes the stayers to their
//     places and the movers' state, compacted, to a buffer; the mover pass
//     writes the movers in their sorted order from that buffer (or from
//     their old slots past its end).
// The result is the same stable order as a full sort of the keys.
#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "sort_view.h"

namespace ffpic {

constexpr int kTile = 1 << kTileShift;      // slots per classify tile (8 per thread)
constexpr int kTileWords = kTile / 64;      // 64-slot words per tile
constexpr int kGroup = 1 << kGroupShift;    // tiles per group of the tile scan
constexpr int kRsItems = 16;                // pairs per thread of a radix tile
constexpr int kRsTile = 256 * kRsItems;     // pairs per radix tile
constexpr int kMoverBlocks = 8192;          // blocks of the passes over the movers
constexpr int kRsBlocks = 2048;             // blocks of a radix pass

#define HCHK_SORT(x)                                                                    \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) throw std::runtime_error(hipGetErrorString(e_));          \
    } while (0)

// ---------------------------------------------------------------------------
// small device helpers

__device__ __forceinline__ uint64_t lanes_below() {
    return (1ull << (threadIdx.x & 63)) - 1ull;
}

// exclusive scan of one value per thread over a block of 256 threads; the
// block total in *total.  Contains barriers: every thread of the block must
// call it.
__device__ __forceinline__ uint64_t block_scan256(uint64_t v, uint64_t *total) {
    __shared__ uint64_t wt[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wt[w] = x;
    __syncthreads();
    uint64_t pre = 0;
    for (int u = 0; u < w; u++) pre += wt[u];
    *total = wt[0] + wt[1] + wt[2] + wt[3];
    __syncthreads();
    return pre + x - v;
}

// lanes of the wave whose (valid) digit equals this lane's
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t x = __ballot(bit);
        m &= bit ? x : ~x;
    }
    return m;
}

__global__ void k_set_i32(int32_t *p, int32_t v) { p[0] = v; }

// ---------------------------------------------------------------------------
// key pass of the full sort and of the removal without sorting

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
__global__ void k_count_sorted(const int32_t *__restrict__ n_dev, const uint32_t *__restrict__ keys,
                               uint32_t dead, int32_t *__restrict__ nalive,
                               int32_t *__restrict__ nslots, int32_t *__restrict__ nsorted) {
    int lo = 0, hi = n_dev[0];
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

__global__ void k_copy_u32(const int32_t *__restrict__ n_dev, const uint32_t *__restrict__ src,
                           uint32_t *__restrict__ dst) {
    const int n = n_dev[0];
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
        dst[q] = src[q];
}

__global__ void k_zero_i32(int32_t *p, int n) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0;
}

void zero_counters(ffpic_ctx *c, int32_t *p, int n) {
    hipLaunchKernelGGL(k_zero_i32, dim3((n + 63) / 64), dim3(64), 0, c->stream, p, n);
}

// ---------------------------------------------------------------------------
// exclusive scan of n int32 values (n known on the host), three launches:
// block sums, a scan of the block sums, the scan of each block

__global__ void __launch_bounds__(256) k_scan_sums(const int32_t *__restrict__ in, int n,
                                                   int32_t *__restrict__ part) {
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    int s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++)
        if (base + u < n) s += in[base + u];
    uint64_t tot;
    (void)block_scan256((uint64_t)(uint32_t)s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = (int32_t)tot;
}

__global__ void __launch_bounds__(256) k_scan_part(int32_t *__restrict__ part, int nb) {
    uint64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int base = b0 + threadIdx.x * 4;
        int32_t v[4];
        uint64_t s = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            v[u] = base + u < nb ? part[base + u] : 0;
            s += (uint32_t)v[u];
        }
        uint64_t tot;
        uint64_t ex = block_scan256(s, &tot) + carry;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (base + u < nb) part[base + u] = (int32_t)ex;
            ex += (uint32_t)v[u];
        }
        carry += tot;
    }
}

__global__ void __launch_bounds__(256) k_scan_apply(const int32_t *__restrict__ in, int n,
                                                    const int32_t *__restrict__ part,
                                                    int32_t *__restrict__ out) {
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    int32_t v[4];
    uint64_t s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        v[u] = base + u < n ? in[base + u] : 0;
        s += (uint32_t)v[u];
    }
    uint64_t tot;
    uint64_t ex = block_scan256(s, &tot) + (uint32_t)part[blockIdx.x];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        if (base + u < n) out[base + u] = (int32_t)ex;
        ex += (uint32_t)v[u];
    }
}

int64_t scan_part_len(int64_t n) { return (n + 1023) / 1024 + 1; }

void exclusive_scan_i32(ffpic_ctx *c, const int32_t *in, int32_t *out, int64_t n) {
    if (n <= 0) return;
    const int nb = (int)((n + 1023) / 1024);
    if (scan_part_len(n) > c->scan_part_n) throw std::runtime_error("scan scratch too small");
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, c->stream, in, (int)n, c->scan_part);
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(256), 0, c->stream, c->scan_part, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(256), 0, c->stream, in, (int)n, c->scan_part,
                       out);
    FFPIC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// LSD radix sort of (key, value) pairs; the count is read on the device

// digit histogram of every tile (tiles strided over the blocks)
__global__ void __launch_bounds__(256) k_rs_hist(const uint32_t *__restrict__ keys,
                                                 const int32_t *__restrict__ n_dev, int shift,
                                                 uint32_t *__restrict__ hist, int stride) {
    const int n = n_dev[0];
    const int nt = (n + kRsTile - 1) / kRsTile;
    __shared__ uint32_t h[256];
    const uint64_t below = lanes_below();
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int i0 = t * kRsTile;
        h[threadIdx.x] = 0;
        __syncthreads();
        for (int r = 0; r < kRsItems; r++) {
            const int i = i0 + r * 256 + threadIdx.x;
            const bool valid = i < n;
            const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
            const uint64_t peers = digit_peers(d, valid);
            if (valid && (peers & below) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
        }
        __syncthreads();
        hist[(size_t)threadIdx.x * stride + t] = h[threadIdx.x];
    }
}

// exclusive scan over the tiles of one digit (one block per digit), in
// place; the digit's total in dtot
__global__ void __launch_bounds__(256) k_rs_scan(uint32_t *__restrict__ hist, int stride,
                                                 const int32_t *__restrict__ n_dev,
                                                 uint32_t *__restrict__ dtot) {
    const int nt = (n_dev[0] + kRsTile - 1) / kRsTile;
    uint32_t *row = hist + (size_t)blockIdx.x * stride;
    uint64_t carry = 0;
    for (int t0 = 0; t0 < nt; t0 += 1024) {
        const int base = t0 + threadIdx.x * 4;
        uint32_t v[4];
        uint64_t s = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            v[u] = base + u < nt ? row[base + u] : 0u;
            s += v[u];
        }
        uint64_t tot;
        uint64_t ex = block_scan256(s, &tot) + carry;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            if (base + u < nt) row[base + u] = (uint32_t)ex;
            ex += v[u];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = (uint32_t)carry;
}

// stable scatter (tiles strided over the blocks): a pair's place is the
// digit's base over all tiles, plus the earlier tiles' pairs of that digit,
// plus the pairs of the same digit before it in its tile (rounds of 256 in
// order; inside a round the earlier waves, then the lower lanes of its own
// wave)
__global__ void __launch_bounds__(256) k_rs_scatter(
    const uint32_t *__restrict__ ik, const uint32_t *__restrict__ iv,
    uint32_t *__restrict__ ok, uint32_t *__restrict__ ov, const int32_t *__restrict__ n_dev,
    int shift, const uint32_t *__restrict__ hist, int stride, const uint32_t *__restrict__ dtot) {
    const int n = n_dev[0];
    const int nt = (n + kRsTile - 1) / kRsTile;
    if ((int)blockIdx.x >= nt) return;
    __shared__ uint32_t base[256], run[256], wc[4][256];
    const int tid = threadIdx.x, w = tid >> 6;
    uint64_t tot;
    const uint32_t dbase = (uint32_t)block_scan256(dtot[tid], &tot);
    const uint64_t below = lanes_below();
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int i0 = t * kRsTile;
        base[tid] = dbase + hist[(size_t)tid * stride + t];
        run[tid] = 0;
#pragma unroll
        for (int u = 0; u < 4; u++) wc[u][tid] = 0;
        uint32_t k[kRsItems], v[kRsItems];
#pragma unroll
        for (int r = 0; r < kRsItems; r++) {
            const int i = i0 + r * 256 + tid;
            k[r] = i < n ? ik[i] : 0u;
            v[r] = i < n ? iv[i] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsItems; r++) {
            const bool valid = i0 + r * 256 + tid < n;
            const uint32_t d = (k[r] >> shift) & 255u;
            const uint64_t peers = digit_peers(d, valid);
            if (valid && (peers & below) == 0) wc[w][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            if (valid) {
                uint32_t off = run[d] + (uint32_t)__popcll(peers & below);
                for (int u = 0; u < w; u++) off += wc[u][d];
                const uint32_t dst = base[d] + off;
                ok[dst] = k[r];
                ov[dst] = v[r];
            }
            __syncthreads();
            run[tid] += wc[0][tid] + wc[1][tid] + wc[2][tid] + wc[3][tid];
#pragma unroll
            for (int u = 0; u < 4; u++) wc[u][tid] = 0;
            __syncthreads();
        }
    }
}

struct Pairs {
    uint32_t *k, *v;
};

// sorts the n_dev[0] <= nmax pairs of A by the low `bits` bits of the key;
// B is the second buffer.  Returns the buffer that holds the result.
static Pairs radix_sort(ffpic_ctx *c, Pairs A, Pairs B, const int32_t *n_dev, int64_t nmax,
                        int bits) {
    if (nmax <= 0) return A;
    const int ntile = (int)((nmax + kRsTile - 1) / kRsTile);
    if (ntile > c->rs_stride) throw std::runtime_error("radix histogram too small");
    // the count is known only on the device: a fixed grid strides over the
    // tiles of the largest count
    const int nb = std::min(ntile, kRsBlocks);
    Pairs in = A, out = B;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nb), dim3(256), 0, c->stream, in.k, n_dev, shift,
                           c->rs_hist, c->rs_stride);
        hipLaunchKernelGGL(k_rs_scan, dim3(256), dim3(256), 0, c->stream, c->rs_hist,
                           c->rs_stride, n_dev, c->rs_dtot);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nb), dim3(256), 0, c->stream, in.k, in.v, out.k,
                           out.v, n_dev, shift, c->rs_hist, c->rs_stride, c->rs_dtot);
        FFPIC_LAUNCH_CHECK();
        std::swap(in, out);
    }
    return in;
}

// ---------------------------------------------------------------------------
// geometry of the sort

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

// device scratch of the sort: shared by the species where a sort uses it
// only while it runs (radix histograms, count), per species where a
// placement left to the push still needs it after the sort (class words
// and counts, the key offsets of the stayers, the movers' places)
void sort_alloc(ffpic_ctx *c, int64_t maxcap, void *(*dmalloc)(size_t)) {
    c->rs_stride = (int)std::max<int64_t>(1, (maxcap + kRsTile - 1) / kRsTile);
    c->rs_hist = (uint32_t *)dmalloc((size_t)256 * c->rs_stride * 4);
    c->rs_dtot = (uint32_t *)dmalloc(256 * 4);
    c->rs_n = (int32_t *)dmalloc(4);
    const size_t nk1 = (size_t)c->nr * c->nth + 1;
    for (int s = 0; s < c->d.nspec; s++) {
        const int64_t cap = std::max<int64_t>(c->sp[s].cap, 1);
        const int64_t nw = (cap + 63) / 64 + 1;
        const int64_t nt = (cap + kTile - 1) / kTile + 1;
        const int64_t ng = (nt + kGroup - 1) / kGroup + 1;
        c->sort_smask[s] = (uint64_t *)dmalloc((size_t)nw * 8);
        c->sort_mmask[s] = (uint64_t *)dmalloc((size_t)nw * 8);
        c->sort_wsm[s] = (uint32_t *)dmalloc((size_t)nw * 4);
        c->sort_tc[s] = (uint2 *)dmalloc((size_t)nt * 8);
        c->sort_ts[s] = (uint2 *)dmalloc((size_t)nt * 8);
        c->sort_gs[s] = (uint2 *)dmalloc((size_t)ng * 8);
        c->sort_tot[s] = (uint32_t *)dmalloc(4 * 4);
        c->sort_mst[s] = (int32_t *)dmalloc(nk1 * 4);
        if (!c->fp64) c->sort_dest[s] = (int32_t *)dmalloc((size_t)cap * 4);
    }
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

// test hook (outside the step): offsets of the current order, synchronises
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

// ---------------------------------------------------------------------------
// incremental re-sort

struct ClassArgs {
    int nub, nth, nr;
    uint32_t dead;
    const int32_t *nslots, *nsorted;
    const uint8_t *kill;
    const int32_t *offold;                      // cell offsets of the last sort
    unsigned long long *removed;
    // FP32 state: the cell; FP64 state: r, theta and the geometry
    int32_t *cell;
    double *R;
    const double *TH, *rn, *thn;
    double rmin, dlog, dth;
    uint32_t *keys;                             // FP64: key of every slot (out)
    uint64_t *smask, *mmask;
    uint32_t *wsm;
    uint2 *tc;                                  // stayers, movers of each tile
    uint32_t *tot;                              // [2]: the slot count before the sort
    uint32_t *tkey, *tval;                      // movers of each tile, compacted in it
};

// The key a slot had at the last sort is the one whose range of that
// sort's cell offsets holds the slot: a particle keeps its key since then
// exactly when its slot lies in [OFF[key], OFF[key+1]).  Two reads of the
// per-key offsets instead of a stored key per slot (sorted particles of a
// wave mostly share a key, so the reads share cache lines).  lo, hi: the
// key's OFF[key], OFF[key+1]; nold: the slots the last sort ordered.
__device__ __forceinline__ bool in_old_range(int q, int nold, int lo, int hi) {
    return q < nold && lo <= q && q < hi;
}

// key of every slot, the removal of killed particles, the class bits and
// counts, and the movers of the tile compacted in slot order
template <bool FP64>
__global__ void __launch_bounds__(256) k_classify(ClassArgs A) {
    constexpr int K = kTile / 256;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int base = blockIdx.x * kTile;
    const int ns = A.nslots[0], no = A.nsorted[0];
    if (blockIdx.x == 0 && tid == 0) A.tot[2] = (uint32_t)ns;   // for a push that places
    uint32_t key[K];
    int cl[K];
    if (!FP64) {
        // the cells of all K slots, then for every slot its cell's kill flag
        // and its key's old offset range, loaded whether needed or not (a
        // slot without a particle reads those of key 0): with no branch
        // around them, all 3K loads are in flight together instead of one
        // round trip after another
        int cell[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int q = base + k * 256 + tid;
            cell[k] = q < ns ? A.cell[q] : -1;
        }
        uint8_t kf[K];
        int lo[K], hi[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int c = cell[k];
            const uint32_t kk =
                c >= 0 ? (uint32_t)(c >> 16) * (uint32_t)A.nth + (uint32_t)(c & 0xffff) : 0u;
            key[k] = kk;
            kf[k] = A.kill[kk];
            lo[k] = A.offold[kk];
            hi[k] = A.offold[kk + 1];
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int q = base + k * 256 + tid;
            const bool live = cell[k] >= 0;
            const bool killed = live && kf[k] != 0;
            if (killed) A.cell[q] = -1;
            if (!live || killed) key[k] = A.dead;
            cl[k] = key[k] >= A.dead ? 0 : (in_old_range(q, no, lo[k], hi[k]) ? 1 : 2);
            count_wave(&A.removed[1], killed);
        }
    } else {
        // the positions of all K slots, their cells, then (as in the FP32
        // branch) the kill flags and old offset ranges, loaded unconditionally
        double r[K], th[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int q = base + k * 256 + tid;
            r[k] = q < ns ? A.R[q] : -1.0;
            th[k] = q < ns ? A.TH[q] : 0.0;
        }
        int cix[K];                                 // i * nth + j, -1: no particle
#pragma unroll
        for (int k = 0; k < K; k++) {
            cix[k] = -1;
            if (r[k] > 0.0) {
                int i, j;
                double a, b;
                locate64(A.nr, A.nth, A.rmin, A.dlog, A.dth, A.rn, A.thn, r[k], th[k], i, j, a, b);
                cix[k] = i * A.nth + j;
            }
        }
        uint8_t kf[K];
        int lo[K], hi[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const uint32_t kk = cix[k] >= 0 ? (uint32_t)cix[k] : 0u;
            kf[k] = A.kill[kk];
            lo[k] = A.offold[kk];
            hi[k] = A.offold[kk + 1];
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int q = base + k * 256 + tid;
            const bool live = cix[k] >= 0;
            const bool killed = live && kf[k] != 0;
            if (killed) A.R[q] = -1.0;
            key[k] = live && !killed ? (uint32_t)cix[k] : A.dead;
            if (q < A.nub) A.keys[q] = key[k];
            cl[k] = key[k] >= A.dead ? 0 : (in_old_range(q, no, lo[k], hi[k]) ? 1 : 2);
            count_wave(&A.removed[1], killed);
        }
    }
    // the tile's words are staged in LDS and written by 16 lanes at once
    __shared__ uint64_t wmask[2][kTileWords];
    __shared__ uint32_t wpre[2][kTileWords];
    uint64_t mm[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint64_t sm = __ballot(cl[k] == 1);
        mm[k] = __ballot(cl[k] == 2);
        if (lane == 0) {
            wmask[0][k * 4 + w] = sm;
            wmask[1][k * 4 + w] = mm[k];
        }
    }
    __syncthreads();
    const int nwu = (A.nub + 63) >> 6;
    if (tid < kTileWords) {
        uint32_t ps = 0, pm = 0;
        for (int u = 0; u < tid; u++) {
            ps += (uint32_t)__popcll(wmask[0][u]);
            pm += (uint32_t)__popcll(wmask[1][u]);
        }
        wpre[0][tid] = ps;
        wpre[1][tid] = pm;
        const int gw = (base >> 6) + tid;
        if (gw < nwu) {
            A.smask[gw] = wmask[0][tid];
            A.mmask[gw] = wmask[1][tid];
            A.wsm[gw] = ps | (pm << 16);
        }
        if (tid == kTileWords - 1)
            A.tc[blockIdx.x] = make_uint2(ps + (uint32_t)__popcll(wmask[0][tid]),
                                          pm + (uint32_t)__popcll(wmask[1][tid]));
    }
    __syncthreads();
    const uint64_t below = lanes_below();
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (cl[k] == 2) {
            const int r = (int)wpre[1][k * 4 + w] + (int)__popcll(mm[k] & below);
            A.tkey[base + r] = key[k];
            A.tval[base + r] = (uint32_t)(base + k * 256 + tid);
        }
    }
}

// exclusive scan of the tile counts inside each group of kGroup tiles; the
// group totals go to gs (scanned by k_group_scan)
__global__ void __launch_bounds__(256) k_tile_scan(const uint2 *__restrict__ tc, int ntile,
                                                   uint2 *__restrict__ ts, uint2 *__restrict__ gs) {
    const int t0 = blockIdx.x * kGroup + threadIdx.x * 4;
    uint2 v[4];
    uint64_t s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        v[u] = t0 + u < ntile ? tc[t0 + u] : make_uint2(0u, 0u);
        s += (uint64_t)v[u].x | ((uint64_t)v[u].y << 32);
    }
    uint64_t tot;
    uint64_t ex = block_scan256(s, &tot);
#pragma unroll
    for (int u = 0; u < 4; u++) {
        if (t0 + u < ntile) ts[t0 + u] = make_uint2((uint32_t)ex, (uint32_t)(ex >> 32));
        ex += (uint64_t)v[u].x | ((uint64_t)v[u].y << 32);
    }
    if (threadIdx.x == 0) gs[blockIdx.x] = make_uint2((uint32_t)tot, (uint32_t)(tot >> 32));
}

// exclusive scan of the group totals (at most 1024 groups), and the totals
__global__ void __launch_bounds__(256) k_group_scan(uint2 *__restrict__ gs, int ngroup,
                                                    uint32_t *__restrict__ tot) {
    const int g0 = threadIdx.x * 4;
    uint2 v[4];
    uint64_t s = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        v[u] = g0 + u < ngroup ? gs[g0 + u] : make_uint2(0u, 0u);
        s += (uint64_t)v[u].x | ((uint64_t)v[u].y << 32);
    }
    uint64_t all;
    uint64_t ex = block_scan256(s, &all);
#pragma unroll
    for (int u = 0; u < 4; u++) {
        if (g0 + u < ngroup) gs[g0 + u] = make_uint2((uint32_t)ex, (uint32_t)(ex >> 32));
        ex += (uint64_t)v[u].x | ((uint64_t)v[u].y << 32);
    }
    if (threadIdx.x == 0) {
        tot[0] = (uint32_t)all;
        tot[1] = (uint32_t)(all >> 32);
    }
}

// the movers of every tile into one array, in slot order (one wave a tile)
__global__ void __launch_bounds__(256) k_movers_dense(int ntile, const uint2 *__restrict__ tc,
                                                      const uint2 *__restrict__ ts,
                                                      const uint2 *__restrict__ gs,
                                                      const uint32_t *__restrict__ tkey,
                                                      const uint32_t *__restrict__ tval,
                                                      uint32_t *__restrict__ mk,
                                                      uint32_t *__restrict__ mv) {
    const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= ntile) return;
    const int cnt = (int)tc[t].y;
    const uint32_t b = gs[t / kGroup].y + ts[t].y;
    for (int i = lane; i < cnt; i += 64) {
        mk[b + i] = tkey[(size_t)t * kTile + i];
        mv[b + i] = tval[(size_t)t * kTile + i];
    }
}

// first index in [lo, hi) whose value is >= x
__device__ __forceinline__ int lower_bound_u32(const uint32_t *a, int lo, int hi, uint32_t x) {
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// movers per key: the first mover of each run of equal (sorted) keys
// writes the run's length; keys without movers keep the zero that
// k_key_offsets leaves behind
__global__ void __launch_bounds__(256) k_mover_runs(const uint32_t *__restrict__ tot,
                                                    const uint32_t *__restrict__ mk,
                                                    int32_t *__restrict__ cnt) {
    const int m = (int)tot[1];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const uint32_t key = mk[j];
        if (j > 0 && mk[j - 1] == key) continue;
        // end of the run, by galloping then bisection
        int step = 1;
        while (j + step < m && mk[j + step] == key) step <<= 1;
        const int hi = lower_bound_u32(mk, j + (step >> 1), min(j + step, m), key + 1u);
        cnt[key] = hi - j;
    }
}

// per key k, from the exclusive scan of the mover counts (the block sums
// scanned by k_scan_part): moff[k] = movers with key < k; mst[k] = moff[k]
// plus the movers of key k from a slot below OFF[k]; the new offsets
// SB(OFF[k]) + moff[k]; the new live count.  Clears the counts for the
// next sort.
__global__ void __launch_bounds__(256) k_key_offsets(
    int nkeys, ClassView V, const uint32_t *__restrict__ mv, const int32_t *__restrict__ offold,
    int32_t *__restrict__ cnt, const int32_t *__restrict__ part, int32_t *__restrict__ mst,
    int32_t *__restrict__ offnew, int32_t *__restrict__ nalive, int32_t *__restrict__ nslots,
    int32_t *__restrict__ nsorted) {
    const int n = nkeys + 1;
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    int32_t cu[4];
    uint64_t sum = 0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        cu[u] = base + u < n ? cnt[base + u] : 0;
        sum += (uint32_t)cu[u];
    }
    // the four keys' old offsets, then the stayer counts before them, each
    // loaded for all four at once (a key past the last reads the last key's;
    // an offset at or past the slot bound reads slot nub - 1's words and
    // takes the stayer total instead): behind a branch per key, each load
    // waited for the one before
    int x[4];
#pragma unroll
    for (int u = 0; u < 4; u++) x[u] = offold[min(base + u, n - 1)];
    uint32_t sb[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int xs = min(x[u], V.nub - 1);
        const int wd = xs >> 6;
        const uint64_t below = (1ull << (xs & 63)) - 1ull;
        sb[u] = V.gs[xs >> (kTileShift + kGroupShift)].x + V.ts[xs >> kTileShift].x +
                (V.wsm[wd] & 0xffffu) + (uint32_t)__popcll(V.smask[wd] & below);
    }
    const uint32_t stot = V.tot[0];
    uint64_t tot;
    uint32_t lo = (uint32_t)(block_scan256(sum, &tot) + (uint32_t)part[blockIdx.x]);
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int k = base + u;
        if (k >= n) break;
        const uint32_t hi = lo + (uint32_t)cu[u];
        const int v = (int)((x[u] >= V.nub ? stot : sb[u]) + lo);
        offnew[k] = v;
        if (k == nkeys) {
            nalive[0] = v;
            nslots[0] = v;
            nsorted[0] = v;
        } else {
            // the movers of key k are in slot order
            mst[k] = cu[u] ? lower_bound_u32(mv, (int)lo, (int)hi, (uint32_t)x[u]) : (int)lo;
            if (cu[u]) cnt[k] = 0;
        }
        lo = hi;
    }
}

// stayers to their places; movers' state to the compact buffer.  Each
// thread takes two slots 256 apart, so twice the state loads are in flight
template <typename T, int NA, bool FP64>
__device__ __forceinline__ void place_slot(const ClassView &V, int nth, const uint32_t *keys,
                                           const int32_t *mst, int32_t *perm, const PtrSet<T, NA> &P,
                                           T *cbuf, int64_t cn, int q, const T (&v)[NA]) {
    const int wd = q >> 6;
    const uint64_t bit = 1ull << (q & 63);
    const uint64_t sm = V.smask[wd], mm = V.mmask[wd];
    if (sm & bit) {
        uint32_t key;
        if (FP64) {
            key = keys[q];
        } else {
            const int cell = (int)v[0];
            key = (uint32_t)(cell >> 16) * (uint32_t)nth + (uint32_t)(cell & 0xffff);
        }
        const uint32_t d = stayers_before(V, q) + (uint32_t)mst[key];
#pragma unroll
        for (int a = 0; a < NA; a++) P.dst[a][d] = v[a];
        if (perm) perm[d] = q;
    } else if (mm & bit) {
        const int64_t im = movers_before(V, q);
        if (im < cn) {
#pragma unroll
            for (int a = 0; a < NA; a++) cbuf[(size_t)a * (size_t)cn + (size_t)im] = v[a];
        }
    }
}

template <typename T, int NA, bool FP64>
__global__ void __launch_bounds__(256) k_place_stayers(
    ClassView V, int nth, const uint32_t *__restrict__ keys, const int32_t *__restrict__ mst,
    int32_t *__restrict__ perm, PtrSet<T, NA> P, T *__restrict__ cbuf, int64_t cn) {
    // slots past the live ones, dead slots and killed particles have
    // neither bit (and are read for nothing); the state is read before the
    // class words so that its loads overlap theirs
    const int q0 = blockIdx.x * 512 + threadIdx.x, q1 = q0 + 256;
    T v0[NA], v1[NA];
#pragma unroll
    for (int a = 0; a < NA; a++) {
        v0[a] = q0 < V.nub ? P.src[a][q0] : T(0);
        v1[a] = q1 < V.nub ? P.src[a][q1] : T(0);
    }
    if (q0 < V.nub) place_slot<T, NA, FP64>(V, nth, keys, mst, perm, P, cbuf, cn, q0, v0);
    if (q1 < V.nub) place_slot<T, NA, FP64>(V, nth, keys, mst, perm, P, cbuf, cn, q1, v1);
}

// movers in their sorted order: rank j (key k, slot q) goes to
// j + SB(clamp(q, OFF[k], OFF[k+1]))
template <typename T, int NA>
__global__ void __launch_bounds__(256) k_place_movers(
    ClassView V, const uint32_t *__restrict__ mk, const uint32_t *__restrict__ mv,
    const int32_t *__restrict__ offold, int32_t *__restrict__ perm, PtrSet<T, NA> P,
    const T *__restrict__ cbuf, int64_t cn) {
    const int m = (int)V.tot[1];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const uint32_t key = mk[j];
        const int q = (int)mv[j];
        const int lo = offold[key], hi = offold[key + 1];
        const int cq = q < lo ? lo : (q > hi ? hi : q);
        const uint32_t d = (uint32_t)j + stayers_before(V, cq);
        const int64_t im = movers_before(V, q);
        T v[NA];
        if (im < cn) {
#pragma unroll
            for (int a = 0; a < NA; a++) v[a] = cbuf[(size_t)a * (size_t)cn + (size_t)im];
        } else {
#pragma unroll
            for (int a = 0; a < NA; a++) v[a] = P.src[a][q];
        }
#pragma unroll
        for (int a = 0; a < NA; a++) P.dst[a][d] = v[a];
        if (perm) perm[d] = q;
    }
}

// For a push that places the sort: the place of the particle in every
// slot, written by slot.  Movers first (from their ranks), then the other
// slots: a stayer's place as in k_place_stayers, -1 for a slot that holds no
// particle of the new order.  Both write the permutation.
__global__ void __launch_bounds__(256) k_mover_dest(ClassView V, const uint32_t *__restrict__ mk,
                                                    const uint32_t *__restrict__ mv,
                                                    const int32_t *__restrict__ offold,
                                                    int32_t *__restrict__ dest,
                                                    int32_t *__restrict__ perm) {
    const int m = (int)V.tot[1];
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
        const uint32_t key = mk[j];
        const int q = (int)mv[j];
        const int lo = offold[key], hi = offold[key + 1];
        const int cq = q < lo ? lo : (q > hi ? hi : q);
        const uint32_t d = (uint32_t)j + stayers_before(V, cq);
        dest[q] = (int32_t)d;
        if (perm) perm[d] = q;
    }
}

// eight slots per thread, 256 apart: the loads of all eight cells, then of
// their keys' mover counts (for every slot, a slot without a particle reading
// key 0's, so that no branch separates them), are in flight together.  The
// 64 slots of a wave are one class word, so the words, their counts and the
// tile and group counts are read once per wave with scalar loads.
constexpr int kDestSlots = 8;

__global__ void __launch_bounds__(256) k_stayer_dest(ClassView V, int nth,
                                                     const int32_t *__restrict__ cell,
                                                     const int32_t *__restrict__ mst,
                                                     int32_t *__restrict__ dest,
                                                     int32_t *__restrict__ perm) {
    const int lane = threadIdx.x & 63;
    // first slot of this wave in round k: wave-uniform
    const int wbase = __builtin_amdgcn_readfirstlane(
        (int)(blockIdx.x * (256 * kDestSlots) + (threadIdx.x & ~63u)));
    const uint64_t below = (1ull << lane) - 1ull;
    int c[kDestSlots];
#pragma unroll
    for (int k = 0; k < kDestSlots; k++) {
        const int q = wbase + k * 256 + lane;
        c[k] = q < V.nub ? cell[q] : -1;
    }
    int32_t ms[kDestSlots];
#pragma unroll
    for (int k = 0; k < kDestSlots; k++) {
        const uint32_t key =
            c[k] >= 0 ? (uint32_t)(c[k] >> 16) * (uint32_t)nth + (uint32_t)(c[k] & 0xffff) : 0u;
        ms[k] = mst[key];
    }
    int32_t d[kDestSlots];
    bool mover[kDestSlots];
#pragma unroll
    for (int k = 0; k < kDestSlots; k++) {
        const int q0 = wbase + k * 256;             // a whole class word
        d[k] = -1;
        mover[k] = false;
        if (q0 < V.nub) {
            const int wd = q0 >> 6;
            const uint64_t sm = V.smask[wd], mm = V.mmask[wd];
            mover[k] = ((mm >> lane) & 1ull) != 0;
            if ((sm >> lane) & 1ull) {
                const uint32_t before = V.gs[q0 >> (kTileShift + kGroupShift)].x +
                                        V.ts[q0 >> kTileShift].x + (V.wsm[wd] & 0xffffu) +
                                        (uint32_t)__popcll(sm & below);
                d[k] = (int32_t)(before + (uint32_t)ms[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kDestSlots; k++) {
        const int q = wbase + k * 256 + lane;
        if (q >= V.nub || mover[k]) continue;       // a mover: placed by its rank
        if (d[k] >= 0 && perm) perm[d[k]] = q;
        dest[q] = d[k];
    }
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

static int32_t *perm_out(ffpic_ctx *c, int s) {
    c->perm_valid[s] = c->record_perm && c->perm[s];
    return c->perm_valid[s] ? c->perm[s] : nullptr;
}

// full sort: key pass, radix sort of all (key, slot) pairs, gather; then the
// sorted keys and cell offsets are kept for the next (incremental) sort
static void sort_full(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    const int nub = (int)S.nub;
    const uint32_t dead = dead_key(c);
    key_pass(c, s, dead);
    hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(1), 0, c->stream, c->rs_n, nub);
    const Pairs R = radix_sort(c, Pairs{c->keys[0], c->vals[0]}, Pairs{c->keys[1], c->vals[1]},
                               c->rs_n, nub, sort_key_bits(c));
    int32_t *nal = c->nalive + s;
    hipLaunchKernelGGL(k_count_sorted, dim3(1), dim3(1), 0, c->stream, c->rs_n, R.k, dead, nal,
                       c->nslots + s, c->nsorted + s);
    const int nb = std::max(1, std::min((nub + 255) / 256, 65536));
    if (c->fp64) {
        hipLaunchKernelGGL((k_gather_set<uint64_t, 5>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, R.v, (state_ptrs<uint64_t, 5>(S)));
    } else {
        hipLaunchKernelGGL((k_gather_set<uint32_t, 6>), dim3(nb), dim3(256), 0, c->stream, nub,
                           nal, R.v, (state_ptrs<uint32_t, 6>(S)));
    }
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
    // the sorted keys and their cell offsets, for the next sort
    const int t = c->sort_cur[s];
    if (int32_t *perm = perm_out(c, s))
        hipLaunchKernelGGL(k_copy_u32, dim3(nb), dim3(256), 0, c->stream, nal, R.v,
                           (uint32_t *)perm);
    const int nkeys = c->nr * c->nth;
    hipLaunchKernelGGL(k_offsets_dev, dim3((nkeys + 1 + 255) / 256), dim3(256), 0, c->stream, nal,
                       R.k, nkeys, c->soff[s][t]);
    FFPIC_LAUNCH_CHECK();
    c->sort_valid[s] = true;
}

// incremental sort (see the header comment); requires the keys and offsets
// of the previous sort of this species
static void sort_incremental(ffpic_ctx *c, int s, bool defer) {
    ffpic::Species &S = c->sp[s];
    const int nub = (int)S.nub;
    const uint32_t dead = dead_key(c);
    const int nkeys = c->nr * c->nth;
    const int t = c->sort_cur[s];
    const int ntile = (nub + kTile - 1) / kTile;
    const int ngroup = (ntile + kGroup - 1) / kGroup;
    if (ngroup > 1024) throw std::runtime_error("more slots than the sort handles");

    ClassArgs A{};
    A.nub = nub;
    A.nth = c->nth;
    A.nr = c->nr;
    A.dead = dead;
    A.nslots = c->nslots + s;
    A.nsorted = c->nsorted + s;
    A.kill = c->kill;
    A.offold = c->soff[s][t];
    A.removed = c->removed + 4 * s;
    A.smask = c->sort_smask[s];
    A.mmask = c->sort_mmask[s];
    A.wsm = c->sort_wsm[s];
    A.tc = c->sort_tc[s];
    A.tot = c->sort_tot[s];
    // the movers of each tile go to the second radix buffer, which is free
    // until the movers have been made dense
    A.tkey = c->keys[1];
    A.tval = c->vals[0];
    if (c->fp64) {
        A.R = (double *)S.cur[0];
        A.TH = (const double *)S.cur[1];
        A.rn = c->dtab64[T_RN];
        A.thn = c->dtab64[T_THN];
        A.rmin = c->d.rmin;
        A.dlog = c->dlog;
        A.dth = c->dth;
        A.keys = c->keys[0];
        hipLaunchKernelGGL(k_classify<true>, dim3(ntile), dim3(256), 0, c->stream, A);
    } else {
        A.cell = (int32_t *)S.cur[0];
        hipLaunchKernelGGL(k_classify<false>, dim3(ntile), dim3(256), 0, c->stream, A);
    }
    hipLaunchKernelGGL(k_tile_scan, dim3(ngroup), dim3(256), 0, c->stream, c->sort_tc[s], ntile,
                       c->sort_ts[s], c->sort_gs[s]);
    hipLaunchKernelGGL(k_group_scan, dim3(1), dim3(256), 0, c->stream, c->sort_gs[s], ngroup,
                       c->sort_tot[s]);
    FFPIC_LAUNCH_CHECK();
    const Pairs dense{c->vals[1], c->sort_aux}, spare{c->keys[1], c->vals[0]};
    hipLaunchKernelGGL(k_movers_dense, dim3((ntile + 3) / 4), dim3(256), 0, c->stream, ntile,
                       c->sort_tc[s], c->sort_ts[s], c->sort_gs[s], A.tkey, A.tval, dense.k, dense.v);
    FFPIC_LAUNCH_CHECK();
    // the mover count is tot[1], on the device
    const int32_t *m_dev = (const int32_t *)(c->sort_tot[s] + 1);
    const Pairs M = radix_sort(c, dense, spare, m_dev, nub, sort_key_bits(c));

    ClassView V{nub, c->sort_smask[s], c->sort_mmask[s], c->sort_wsm[s], c->sort_ts[s], c->sort_gs[s],
                c->sort_tot[s]};
    const int32_t *offold = c->soff[s][t];
    int32_t *offnew = c->soff[s][1 - t];
    // movers per key, their exclusive scan, and the per-key pass
    const int nbk = (int)((nkeys + 1 + 1023) / 1024);
    const int nbm = std::max(1, std::min((nub + 255) / 256, kMoverBlocks));
    if (scan_part_len(nkeys + 1) > c->scan_part_n) throw std::runtime_error("scan scratch too small");
    hipLaunchKernelGGL(k_mover_runs, dim3(nbm), dim3(256), 0, c->stream, c->sort_tot[s], M.k,
                       c->sort_kcnt);
    hipLaunchKernelGGL(k_scan_sums, dim3(nbk), dim3(256), 0, c->stream, c->sort_kcnt, nkeys + 1,
                       c->scan_part);
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(256), 0, c->stream, c->scan_part, nbk);
    // reads the old live count (through OFF) before replacing it
    hipLaunchKernelGGL(k_key_offsets, dim3(nbk), dim3(256), 0, c->stream, nkeys, V, M.v, offold,
                       c->sort_kcnt, c->scan_part, c->sort_mst[s], offnew, c->nalive + s,
                       c->nslots + s, c->nsorted + s);
    FFPIC_LAUNCH_CHECK();
    int32_t *perm = perm_out(c, s);
    if (defer) {
        // the next push reads the particles in the old order and writes
        // them in the new one (FP32): it reads where each goes
        hipLaunchKernelGGL(k_mover_dest, dim3(nbm), dim3(256), 0, c->stream, V, M.k, M.v, offold,
                           c->sort_dest[s], perm);
        hipLaunchKernelGGL(k_stayer_dest, dim3((nub + 256 * kDestSlots - 1) / (256 * kDestSlots)),
                           dim3(256), 0, c->stream, V,
                           c->nth, (const int32_t *)S.cur[0], c->sort_mst[s], c->sort_dest[s],
                           perm);
        FFPIC_LAUNCH_CHECK();
        SortPlace &P = c->place[s];
        P.dest = c->sort_dest[s];
        P.cell = (int32_t *)S.alt[0];
        P.a = (float *)S.alt[1];
        P.b = (float *)S.alt[2];
        P.ur = (float *)S.alt[3];
        P.ut = (float *)S.alt[4];
        P.up = (float *)S.alt[5];
        c->sort_pending[s] = true;
        c->sort_cur[s] = 1 - t;
        return;
    }
    const int nbs = (nub + 511) / 512;
    if (c->fp64) {
        auto P = state_ptrs<uint64_t, 5>(S);
        hipLaunchKernelGGL((k_place_stayers<uint64_t, 5, true>), dim3(nbs), dim3(256), 0,
                           c->stream, V, c->nth, c->keys[0], c->sort_mst[s], perm,
                           P, (uint64_t *)c->sort_cbuf, c->sort_cbuf_n);
        hipLaunchKernelGGL((k_place_movers<uint64_t, 5>), dim3(nbm), dim3(256), 0, c->stream, V,
                           M.k, M.v, offold, perm, P, (const uint64_t *)c->sort_cbuf,
                           c->sort_cbuf_n);
    } else {
        auto P = state_ptrs<uint32_t, 6>(S);
        hipLaunchKernelGGL((k_place_stayers<uint32_t, 6, false>), dim3(nbs), dim3(256), 0,
                           c->stream, V, c->nth, nullptr, c->sort_mst[s], perm, P,
                           (uint32_t *)c->sort_cbuf, c->sort_cbuf_n);
        hipLaunchKernelGGL((k_place_movers<uint32_t, 6>), dim3(nbm), dim3(256), 0, c->stream, V,
                           M.k, M.v, offold, perm, P, (const uint32_t *)c->sort_cbuf,
                           c->sort_cbuf_n);
    }
    FFPIC_LAUNCH_CHECK();
    for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
    c->sort_cur[s] = 1 - t;
}

void sort_species(ffpic_ctx *c, int s, bool defer) {
    ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    if (c->sort_valid[s] && c->incremental_sort) sort_incremental(c, s, defer && !c->fp64);
    else sort_full(c, s);
}

}  // namespace ffpic
