// FP32-mixed particle push and charge-conserving deposit.
//
// Particle state (SoA, 24 B): cell = (i << 16) | j (int32, -1 = dead slot),
// a = in-cell offset in log r / dlog, b = in-cell offset in theta / dtheta
// (FP32, in [0, 1)), u_r, u_theta, u_phi (FP32).  Splitting the position
// into an integer cell and a small FP32 offset keeps 2^-24 of a cell of
// resolution anywhere on the grid, where an absolute FP32 coordinate would
// lose several digits at r ~ 100.
//
// Physics as in the FP64 path (Sect. 3, eq. motion with the
// radiation-reaction force g and eq. bperp; Boris rotation; zigzag
// charge-conserving deposit), but the move is evaluated in the particle's
// local frame: the radial and polar displacements are formed from the
// small step itself (a log1p series for the radial one, an arctangent
// series for the polar one), so that no difference of two large FP32
// coordinates is ever taken.  Reciprocals and square roots use the
// hardware approximations (about 1 ulp).
//
// The kernel is bound by VALU issue, so it is written for few instructions
// per particle: the axis parity signs are folded into the interpolation
// weights, the particle state is addressed with 32-bit offsets from uniform
// bases, index products use 24-bit multiplies, and the cross-lane sums are
// DPP row reductions.
//
// Gather: each workgroup takes a contiguous chunk of the (cell-sorted)
// particle array and finds the bounding box of its cells.  It copies the six
// field components over the box, with one node of margin, into an LDS patch
// (interleaved per node), and every particle reads its corner pairs from
// there with one ds_read2 each.  Loads from HBM whose lanes read a few nodes
// each would otherwise saturate the vector-memory address unit.
//
// Deposit: the currents accumulate in a second LDS patch covering the box
// plus the one-cell reach of a step; the patch is then flushed to the FP32
// current arrays in HBM with one global atomic per non-zero entry.
// Particles that stay in their cell are summed across each 16-lane row
// first (DPP), one cell per row and pass, so a sorted wave issues one add
// instruction from 32 lanes (eight sums in each of four rows) per pass
// instead of eight from all 64.  Moves that leave their cell (a few per
// cent of a step) are queued in LDS and deposited after the chunk, so the
// zigzag runs in one wave per chunk rather than in nearly every wave.
// Chunks whose box is too large for the patches (sparse regions) gather
// from HBM through buffer resources and add straight to HBM.
#include <algorithm>
#include <cstddef>
#include <cstring>

#include "device_common.h"

namespace ffpic {

constexpr int kWG = 256;
// particles per thread per chunk (a template parameter, chosen by the
// autotuner among 8, 16 and 32; 16 by default): a chunk of 4096 sorted
// particles spans few cells, so its patches' load and flush are spread over
// many particles
constexpr int kTile = 1024;              // LDS deposit patch entries per component
constexpr int kFld = 512;                // LDS field patch nodes (six components each)
constexpr int kQueue = 64;               // queued cell-crossing moves per workgroup
constexpr int kRsrcWord3 = 0x00020000;   // raw dword buffer access (gfx9 family)

struct P32 {
    int nr, nth, ld;
    float dlog, dth, dt, inv_dlog, inv_dth;
    int iabs;                            // r_abs lies in radial cell iabs ...
    float aabs;                          // ... at offset aabs
    const float *rn, *sn, *cn;
    float Q, h, kk;                      // charge, dt omega_b qm / 2, dt K_s
    int ishell;                          // the shell of kept momentum along B ends in
    float ashell;                        // radial cell ishell at offset ashell
};

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
// index products: both factors are grid or patch indices below 2^24 and the
// products stay below 2^32, so the full-rate 24-bit multiply is exact
__device__ __forceinline__ unsigned mul24(int x, unsigned y) { return __umul24((unsigned)x, y); }

// 32-bit element offsets from a uniform base (element index < 2^30)
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + (idx << 2));
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned idx, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + (idx << 2)) = v;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sums eight per-lane values over each 16-lane row, halving the number of
// values at every stage: exchange with lane^1 (keep four), lane^2 (keep
// two), a rotation by four lanes (keep one; it flips bit 2 of the lane and
// keeps bits 0 and 1), and a rotation by eight that adds the other half of
// the row.  Lane l then holds the row sum of value 4*bit0(l) + 2*bit1(l) +
// bit2(l); lanes l and l+8 hold the same sum.  keep[] are the four values a
// lane sums in the first stage (values 4..7 on lanes with bit 0 set, 0..3
// otherwise), pass[] the four its neighbour sums.
__device__ __forceinline__ float row_sum8(const float keep[4], const float pass[4], bool b1,
                                          bool b2) {
    float y[4];
#pragma unroll
    for (int m = 0; m < 4; m++) y[m] = keep[m] + dpp<0xB1>(pass[m]);
    const float z0 = (b1 ? y[2] : y[0]) + dpp<0x4E>(b1 ? y[0] : y[2]);
    const float z1 = (b1 ? y[3] : y[1]) + dpp<0x4E>(b1 ? y[1] : y[3]);
    const float w = (b2 ? z1 : z0) + dpp<0x124>(b2 ? z0 : z1);
    return w + dpp<0x128>(w);
}

// component (0 = J_r, 1 = J_theta, 2 = J_phi) of the row sum a lane holds
// after row_sum8: values 0, 1 are J_r, 2, 3 J_theta, 4..7 J_phi
__device__ __forceinline__ int lane_comp(int lane) {
    const int kq = ((lane & 1) ? 4 : 0) + ((lane & 2) ? 2 : 0) + ((lane & 4) ? 1 : 0);
    return kq < 2 ? 0 : (kq < 4 ? 1 : 2);
}

struct Fields {
    __amdgpu_buffer_rsrc_t er, et, ep, br, bt, bp;
};

// particle state arrays: 32-bit byte offsets (slot * 4) from uniform bases,
// so no 64-bit address is formed per access
struct State {
    int32_t *cell;
    float *a, *b, *ur, *ut, *up;
    __device__ __forceinline__ static float ld(const float *R, unsigned q) { return ldo(R, q); }
    __device__ __forceinline__ static void st(float *R, unsigned q, float v) { sto(R, q, v); }
    __device__ __forceinline__ int ldc(unsigned q) const { return ldo(cell, q); }
    __device__ __forceinline__ void stc(unsigned q, int v) const { sto(cell, q, v); }
};

template <bool LDS>
struct Acc {
    float *tile;     // LDS patch (LDS mode)
    int ti0, tj0, TJ;
    float *g[3];
    int ld;
    __device__ __forceinline__ void add(int comp, int i, int j, float v) const {
        if (LDS) atomicAdd(&tile[comp * kTile + mul24(i - ti0, TJ) + (j - tj0)], v);
        else gadd(reinterpret_cast<float *>(reinterpret_cast<char *>(g[comp]) +
                                            ((mul24(i, ld) + (unsigned)j) << 2)), v);
    }
};

// staggered bilinear interpolation from one buffer: row offset voff (bytes)
// with columns c0 / c1 given as byte offsets, next row via soffset = ld4
__device__ __forceinline__ float bil(__amdgpu_buffer_rsrc_t R, unsigned o0, unsigned o1,
                                     unsigned ld4, float W0, float W1, float wr) {
    // the b32 loads return raw bits
    const float v00 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(R, (int)o0, 0, 0));
    const float v01 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(R, (int)o1, 0, 0));
    const float v10 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(R, (int)o0, (int)ld4, 0));
    const float v11 = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(R, (int)o1, (int)ld4, 0));
    const float lo = v00 * W0 + v01 * W1;
    const float hi = v10 * W0 + v11 * W1;
    return lo + wr * (hi - lo);
}

// zigzag (relay-point) deposit of a move from (x1, y1) in cell (i, j) to
// (x2, y2) in the same frame, ending in cell (i + di, j + dj): the radial and
// polar charge fluxes of the two straight segments, and J_phi at the midpoint
template <bool LDS>
__device__ __forceinline__ void zigzag(const P32 &p, const Acc<LDS> &acc, int i, int j, int di,
                                       int dj, float x1, float y1, float x2, float y2, float qv) {
    const int nth = p.nth;
    const int i2 = i + di, j2 = j + dj;
    const float xr = fminf((float)min(di, 0) + 1.f, fmaxf((float)max(di, 0), 0.5f * (x1 + x2)));
    const float yr = fminf((float)min(dj, 0) + 1.f, fmaxf((float)max(dj, 0), 0.5f * (y1 + y2)));
    const float Q = p.Q;
    const float fx1 = Q * (xr - x1), fy1 = Q * (yr - y1);
    const float fx2 = Q * (x2 - xr), fy2 = Q * (y2 - yr);
    const float wx1 = 0.5f * (x1 + xr), wy1 = 0.5f * (y1 + yr);
    const float wx2 = 0.5f * (xr + x2) - (float)di, wy2 = 0.5f * (yr + y2) - (float)dj;
    acc.add(0, i, j, fx1 * (1.f - wy1));
    acc.add(0, i, j + 1, fx1 * wy1);
    acc.add(1, i, j, fy1 * (1.f - wx1));
    acc.add(1, i + 1, j, fy1 * wx1);
    acc.add(0, i2, j2, fx2 * (1.f - wy2));
    acc.add(0, i2, j2 + 1, fx2 * wy2);
    acc.add(1, i2, j2, fy2 * (1.f - wx2));
    acc.add(1, i2 + 1, j2, fy2 * wx2);
    const float xm = 0.5f * (x1 + x2), ym = 0.5f * (y1 + y2);
    int im = (int)floorf(xm), jm = (int)floorf(ym);
    if (i + im > p.nr - 1) im = p.nr - 1 - i;
    if (j + jm > nth - 1) jm = nth - 1 - j;
    const float wx = xm - (float)im, wy = ym - (float)jm;
    const float qq = Q * qv;
    acc.add(2, i + im, j + jm, qq * (1.f - wx) * (1.f - wy));
    acc.add(2, i + im + 1, j + jm, qq * wx * (1.f - wy));
    acc.add(2, i + im, j + jm + 1, qq * (1.f - wx) * wy);
    acc.add(2, i + im + 1, j + jm + 1, qq * wx * wy);
}

// the same interpolation from the LDS field patch: the node at byte offset
// o of the patch and the next column, and the same pair one patch row (rowB
// bytes) further; the six components of a node are interleaved, so COMP
// selects the word
template <int COMP>
__device__ __forceinline__ float bil_lds(const float *fld, unsigned o, unsigned rowB, float W0,
                                         float W1, float wr) {
    const float *r0 = reinterpret_cast<const float *>(reinterpret_cast<const char *>(fld) + o) + COMP;
    const float *r1 =
        reinterpret_cast<const float *>(reinterpret_cast<const char *>(fld) + o + rowB) + COMP;
    const float lo = r0[0] * W0 + r0[6] * W1;
    const float hi = r1[0] * W0 + r1[6] * W1;
    return lo + wr * (hi - lo);
}

struct Patch {
    const float *fld;    // LDS field patch (LDS mode)
    int fi0, fj0;        // its first row and column
    unsigned rowB;       // bytes per patch row (24 per node)
};

template <bool LDS, bool SHELL, int kPPT, bool PLACE>
__device__ __forceinline__ void push_chunk(const P32 &p, const Fields &F, const Patch &P,
                                           const Acc<LDS> &acc,
                                           int n, int base, int tid, int lane,
                                           const uint8_t *__restrict__ kill, const State &S,
                                           uint32_t *__restrict__ err, int &nkill, int &nstar,
                                           int &nabs, float4 *queue, int *qn, float *kg,
                                           const SortPlace &SP) {
    const int ld = p.ld, nth = p.nth;
    const unsigned ld4 = (unsigned)ld << 2;
    // the next particle's offsets and momentum are loaded one iteration
    // ahead, and the kill flag is applied at the end, so that no state load
    // sits on the latency chain in front of the field gather
    // the deposit value this lane adds after the row reduction: component,
    // radial and polar node offsets from the cell (values 0..7 as below)
    const int rl = lane & 15;
    const bool b0 = rl & 1, b1 = rl & 2, b2 = rl & 4;
    const int kq = (b0 ? 4 : 0) + (b1 ? 2 : 0) + (b2 ? 1 : 0);
    const int kcomp = lane_comp(lane);
    const int kdi = (kq == 3 || kq == 5 || kq == 7) ? 1 : 0;
    const int kdj = (kq == 1 || kq == 6 || kq == 7) ? 1 : 0;
    const bool row_lead = (lane & 8) == 0;
    // LDS mode: a cell's key in the current patch is i * TJ + j (unique over
    // the patch's cells), and the entry this lane adds to after a row sum
    // lies kofs entries from it
    const int kofs = LDS ? kcomp * kTile + kdi * acc.TJ + kdj - acc.ti0 * acc.TJ - acc.tj0 : 0;
    float an = 0.f, bn = 0.f, urn = 0.f, utn = 0.f, upn = 0.f;
    int cn = -1, dn = -1;
    if (base + tid < n) {
        const unsigned q0 = (unsigned)(base + tid);
        cn = S.ldc(q0);
        if (PLACE) dn = ldo(SP.dest, q0);
        an = State::ld(S.a, q0);
        bn = State::ld(S.b, q0);
        urn = State::ld(S.ur, q0);
        utn = State::ld(S.ut, q0);
        upn = State::ld(S.up, q0);
    }
#pragma unroll 1
    for (int k = 0; k < kPPT; k++) {
        const unsigned q = (unsigned)(base + k * kWG + tid);
        const int c = cn;
        bool live = c >= 0;
        const int i = c >> 16, j = c & 0xffff;
        // PLACE: the slot's place in the new order (-1: no particle of it)
        const int dq = dn;
        if (PLACE) live = live && dq >= 0;
        const float a = an, b = bn, ur = urn, ut = utn, up = upn;
        cn = -1;
        if (k + 1 < kPPT && (int)(q + kWG) < n) {
            cn = S.ldc(q + kWG);
            if (PLACE) dn = ldo(SP.dest, q + kWG);
            an = State::ld(S.a, q + kWG);
            bn = State::ld(S.b, q + kWG);
            urn = State::ld(S.ur, q + kWG);
            utn = State::ld(S.ut, q + kWG);
            upn = State::ld(S.up, q + kWG);
        }
        const bool killed = live && kill[mul24(i, nth) + (unsigned)j] != 0;
        // The deposit values below are assigned for every kept particle and
        // read only under `simple` / `cross`, which imply that assignment, so
        // they carry no initial value (no register setup on the other paths).
        bool simple = false;       // stays in its cell: 8 adds at fixed offsets
        float s0, s1, s2, s3, s4, s5, s6, s7;
        float rk[4], rp[4];     // the values split for the row reduction
        bool cross = false;        // leaves its cell: general zigzag
        int di, dj;
        float x1, y1, x2, y2, qv;
        if (live) {
            // ---- staggered bilinear gather
            const bool ah = a >= 0.5f, bh = b >= 0.5f;
            int hr = ah ? i : i - 1;
            float wr = ah ? a - 0.5f : a + 0.5f;
            if (hr < 0) { hr = 0; wr = 0.f; }
            if (hr > p.nr - 2) { hr = p.nr - 2; wr = 1.f; }
            const int ht = bh ? j : j - 1;
            const float wt = bh ? b - 0.5f : b + 0.5f;
            // theta weights: node columns (j, j+1); half columns as the pair
            // (pb, pb+1), where a particle within half a cell of an axis
            // reads the one edge column with both weights (the axis ghost
            // equals it, with the sign flipped for the odd components E_th
            // and B_ph)
            const float Wn0 = 1.f - b, Wn1 = b;
            const float Wh0 = 1.f - wt, Wh1 = wt;
            const bool lo_ax = ht < 0, hi_ax = ht > nth - 2;
            int pb = ht;
            float E0 = Wh0, E1 = Wh1, O0 = Wh0, O1 = Wh1;
            if (__ballot(lo_ax || hi_ax) != 0ull) {   // a wave near an axis (uniform)
                pb = lo_ax ? 0 : (hi_ax ? nth - 2 : ht);
                E0 = lo_ax ? Wh0 + Wh1 : (hi_ax ? 0.f : Wh0);
                E1 = lo_ax ? 0.f : (hi_ax ? Wh0 + Wh1 : Wh1);
                O0 = lo_ax ? Wh1 - Wh0 : (hi_ax ? 0.f : Wh0);
                O1 = lo_ax ? 0.f : (hi_ax ? Wh0 - Wh1 : Wh1);
            }
            float esr, est, esp, bsr, bst, bsp;
            if (LDS) {
                // byte offsets in the patch (24 bytes a node, rowB a row)
                const unsigned rowB = P.rowB;
                const unsigned bn = mul24(i - P.fi0, rowB), bh = mul24(hr - P.fi0, rowB);
                const unsigned cn = mul24(j - P.fj0, 24), ch = mul24(pb - P.fj0, 24);
                esr = bil_lds<0>(P.fld, bh + cn, rowB, Wn0, Wn1, wr);
                est = bil_lds<1>(P.fld, bn + ch, rowB, O0, O1, a);
                esp = bil_lds<2>(P.fld, bn + cn, rowB, Wn0, Wn1, a);
                bsr = bil_lds<3>(P.fld, bn + ch, rowB, E0, E1, a);
                bst = bil_lds<4>(P.fld, bh + cn, rowB, Wn0, Wn1, wr);
                bsp = bil_lds<5>(P.fld, bh + ch, rowB, O0, O1, wr);
            } else {
                const unsigned rN = mul24(i, ld), rH = mul24(hr, ld);
                const unsigned on = (rN + j) << 2, hn = (rH + j) << 2;
                const unsigned oh = (rN + pb) << 2, hh = (rH + pb) << 2;
                esr = bil(F.er, hn, hn + 4, ld4, Wn0, Wn1, wr);
                est = bil(F.et, oh, oh + 4, ld4, O0, O1, a);
                esp = bil(F.ep, on, on + 4, ld4, Wn0, Wn1, a);
                bsr = bil(F.br, oh, oh + 4, ld4, E0, E1, a);
                bst = bil(F.bt, hn, hn + 4, ld4, Wn0, Wn1, wr);
                bsp = bil(F.bp, hh, hh + 4, ld4, O0, O1, wr);
            }
            // ---- geometry: theta = theta_j + d (small-angle series), r = r_i exp(a dlog)
            const float d = b * p.dth, d2 = d * d;
            const float sd = d * (1.f - d2 * (1.f / 6.f) * (1.f - d2 * (1.f / 20.f)));
            const float cd = 1.f - 0.5f * d2 * (1.f - d2 * (1.f / 12.f));
            const float snj = ldo(p.sn, (unsigned)j), cnj = ldo(p.cn, (unsigned)j);
            const float st = snj * cd + cnj * sd;
            const float ct = cnj * cd - snj * sd;
            const float xl = a * p.dlog;
            const float r = ldo(p.rn, (unsigned)i) *
                            (1.f + xl * (1.f + xl * (0.5f + xl * (1.f / 6.f + xl * (1.f / 24.f)))));
            // ---- Boris rotation and radiation reaction in the orthonormal
            // basis (r, theta, phi) at the particle: the vector algebra is the
            // same in any right-handed orthonormal basis
            const float h = p.h;
            const float mx = ur + h * esr, my = ut + h * est, mz = up + h * esp;
            const float ig = h * frsq(1.f + mx * mx + my * my + mz * mz);
            const float tx = bsr * ig, ty = bst * ig, tz = bsp * ig;
            const float sf = 2.f * frcp(1.f + tx * tx + ty * ty + tz * tz);
            const float px = mx + (my * tz - mz * ty);
            const float py = my + (mz * tx - mx * tz);
            const float pz = mz + (mx * ty - my * tx);
            const float sx = tx * sf, sy = ty * sf, sz = tz * sf;
            float nr = mx + (py * sz - pz * sy) + h * esr;
            float nt = my + (pz * sx - px * sz) + h * est;
            float np = mz + (px * sy - py * sx) + h * esp;
            // ---- radiation reaction (explicit, time-centred velocity)
            if (p.kk != 0.f) {
                float bx = 0.5f * (ur + nr), by = 0.5f * (ut + nt), bz = 0.5f * (up + np);
                const float gb2 = 1.f + bx * bx + by * by + bz * bz;
                const float igb = frsq(gb2);
                bx *= igb; by *= igb; bz *= igb;
                const float Fx = esr + (by * bsp - bz * bst);
                const float Fy = est + (bz * bsr - bx * bsp);
                const float Fz = esp + (bx * bst - by * bsr);
                const float be = bx * esr + by * est + bz * esp;
                const float bp2 = fmaxf(Fx * Fx + Fy * Fy + Fz * Fz - be * be, 0.f);
                const float gg = gb2 * bp2;
                const float kk = p.kk;
                nr += kk * ((Fy * bsp - Fz * bst) + be * esr - gg * bx);
                nt += kk * ((Fz * bsr - Fx * bsp) + be * est - gg * by);
                np += kk * ((Fx * bst - Fy * bsr) + be * esp - gg * bz);
            }
            if (SHELL && (i < p.ishell || (i == p.ishell && a < p.ashell))) {
                // shell around the star (Sect. 5): drop the momentum across B
                const float b2 = bsr * bsr + bst * bst + bsp * bsp;
                if (b2 > 0.f) {
                    const float ub = (nr * bsr + nt * bst + np * bsp) / b2;
                    nr = ub * bsr; nt = ub * bst; np = ub * bsp;
                }
            }
            const float ivg = frsq(1.f + nr * nr + nt * nt + np * np);   // 1 / gamma
            const float vdt = p.dt * ivg;
            // the new momentum in the local Cartesian frame at azimuth 0
            // (x along the cylindrical radius, y along phi, z along the axis)
            const float nx = nr * st + nt * ct, ny = np, nz = nr * ct - nt * st;
            const float dx = nx * vdt, dy = ny * vdt, dz = nz * vdt;
            // ---- move in the local frame
            const float w = r * st;
            const float xx = w + dx;
            const float w2 = __builtin_amdgcn_sqrtf(xx * xx + dy * dy);
            const float den = w2 + w;
            const float dw = den > 0.f ? (2.f * w * dx + dx * dx + dy * dy) * frcp(den) : 0.f;
            const float drr = dw * st + dz * ct;
            const float dtt = dw * ct - dz * st;
            const float ir = frcp(r);
            const float yv = drr * ir, zv = dtt * ir;
            const float arg = yv * (2.f + yv) + zv * zv;       // (r'/r)^2 - 1
            const float sq = arg * frcp(2.f + arg);            // log1p(x) = 2 atanh(x / (2 + x))
            const float sq2 = sq * sq;
            const float dxi = sq * (1.f + sq2 * (1.f / 3.f + sq2 * (1.f / 5.f))) * p.inv_dlog;
            const float tq = dtt * frcp(r + drr);
            const float tq2 = tq * tq;
            const float dthe = tq * (1.f - tq2 * (1.f / 3.f - tq2 * (1.f / 5.f)));
            const float iw2 = w2 > 0.f ? frcp(w2) : 0.f;
            const float cp = w2 > 0.f ? xx * iw2 : 1.f;
            const float sp = dy * iw2;
            const float rx = cp * nx + sp * ny, ry = -sp * nx + cp * ny, rz = nz;
            const float dd2 = dthe * dthe;
            const float sdd = dthe * (1.f - dd2 * (1.f / 6.f));
            const float cdd = 1.f - 0.5f * dd2;
            const float st2 = st * cdd + ct * sdd, ct2 = ct * cdd - st * sdd;
            // ---- new cell and offsets (carry)
            float na = a + dxi, nb = b + dthe * p.inv_dth;
            di = (int)floorf(na);
            dj = (int)floorf(nb);
            na -= (float)di;
            nb -= (float)dj;
            if (na >= 1.f) { na -= 1.f; di++; }
            if (nb >= 1.f) { nb -= 1.f; dj++; }
            int i2 = i + di, j2 = j + dj;
            if (j2 < 0) { j2 = 0; nb = 0.f; dj = -j; }
            if (j2 > nth - 1) { j2 = nth - 1; nb = 0.99999994f; dj = j2 - j; }
            const bool cfl = di > 1 || di < -1 || dj > 1 || dj < -1;
            // one test for all five: a NaN or an infinity survives the sum
            const bool finite = __builtin_isfinite(na + nb + rx + ry + rz);
            // a particle in a force-free cell is removed before it moves
            const bool star = !killed && finite && i2 < 0;
            const bool absb = !killed && finite && !star &&
                              (i2 > p.iabs || (i2 == p.iabs && na >= p.aabs));
            const bool keep = !killed && finite && !star && !absb;
            nkill += killed ? 1 : 0;
            nstar += star ? 1 : 0;
            nabs += absb ? 1 : 0;
            if (cfl && !killed) atomicOr(err, FFPIC_ERR_CFL);
            // non-finite state is flagged in the error word and never deposited
            if (!finite && !killed) atomicOr(err, FFPIC_ERR_NONFINITE);
            if (PLACE) {
                const unsigned d = (unsigned)dq;
                sto(SP.cell, d, keep ? ((i2 << 16) | j2) : -1);
                if (keep) {
                    sto(SP.a, d, na);
                    sto(SP.b, d, nb);
                    sto(SP.ur, d, rx * st2 + rz * ct2);
                    sto(SP.ut, d, rx * ct2 - rz * st2);
                    sto(SP.up, d, ry);
                }
            } else {
                S.stc(q, keep ? ((i2 << 16) | j2) : -1);
                if (keep) {
                    State::st(S.a, q, na);
                    State::st(S.b, q, nb);
                    State::st(S.ur, q, rx * st2 + rz * ct2);
                    State::st(S.ut, q, rx * ct2 - rz * st2);
                    State::st(S.up, q, ry);
                }
            }
            x1 = a; y1 = b;
            x2 = (float)di + na;
            y2 = (float)dj + nb;
            qv = ny * ivg;                        // v_phi during the step (before rotation)
            const bool incell = di == 0 && dj == 0;
            simple = keep && !cfl && incell;
            cross = keep && !cfl && !incell;
            // the eight adds of an in-cell move, charge included (computed
            // for every kept particle; used only when it stays in its cell)
            const float ddx = p.Q * (x2 - x1), ddy = p.Q * (y2 - y1);
            const float xm = 0.5f * (x1 + x2), ym = 0.5f * (y1 + y2);
            const float qq = p.Q * qv;
            s1 = ddx * ym;
            s0 = ddx - s1;
            s3 = ddy * xm;
            s2 = ddy - s3;
            s5 = qq * xm;
            s4 = qq - s5;
            s7 = s5 * ym;
            s5 = s5 - s7;
            s6 = s4 * ym;
            s4 = s4 - s6;
            rk[0] = b0 ? s4 : s0; rp[0] = b0 ? s0 : s4;
            rk[1] = b0 ? s5 : s1; rp[1] = b0 ? s1 : s5;
            rk[2] = b0 ? s6 : s2; rp[2] = b0 ? s2 : s6;
            rk[3] = b0 ? s7 : s3; rp[3] = b0 ? s3 : s7;
        }
        // ---- in-cell moves, one cell per 16-lane row and pass: the lanes of
        // a row whose cell is that of the row's first pending lane sum their
        // eight values over the row, and lanes 0..7 of the row add one sum
        // each.  Every pass retires at least the first pending lane of each
        // row, so the loop ends within 16 passes with every in-cell move
        // deposited.  (Sorted particles drift into neighbouring cells between
        // sorts, so a wave holds several cells; the passes with few lanes
        // still cost less than per-lane adds.)
        bool pend = simple;
        const int ckey = LDS ? (int)mul24(i, (unsigned)acc.TJ) + j : c;
#pragma unroll 1
        while (true) {
            const unsigned long long m = __ballot(pend);
            if (m == 0ull) break;
            const unsigned rowm = (unsigned)(m >> (lane & 48)) & 0xffffu;
            const int src = rowm ? (lane & 48) + __builtin_ctz(rowm) : lane;
            const int lc = __shfl(ckey, src, 64);
            const bool part = pend && ckey == lc;
            float pk[4], pp[4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                pk[e] = part ? rk[e] : 0.f;
                pp[e] = part ? rp[e] : 0.f;
            }
            const float v = row_sum8(pk, pp, b1, b2);
            // a row with pending lanes has participants: its leader
            if (row_lead && rowm != 0u) {
                if (LDS) {
                    atomicAdd(&acc.tile[lc + kofs], v);
                } else {
                    const int li = (lc >> 16) + kdi, lj = (lc & 0xffff) + kdj;
                    gadd(reinterpret_cast<float *>(reinterpret_cast<char *>(kg) +
                                                   ((mul24(li, acc.ld) + (unsigned)lj) << 2)), v);
                }
            }
            pend = pend && !part;
        }
        // moves that leave their cell go to the workgroup's queue and are
        // deposited after the chunk, where one wave takes them all instead of
        // every wave that holds one running the zigzag with a few lanes
        const unsigned long long cm = __ballot(cross);
        if (cm != 0ull) {
            int e0 = 0;
            if (lane == 0) e0 = atomicAdd(qn, __popcll(cm));
            e0 = __builtin_amdgcn_readfirstlane(e0);
            if (cross) {
                const int e = e0 + (int)__builtin_amdgcn_mbcnt_hi(
                                       (unsigned)(cm >> 32),
                                       __builtin_amdgcn_mbcnt_lo((unsigned)cm, 0u));
                if (e < kQueue) {
                    queue[2 * e] = make_float4(__int_as_float(c),
                                               __int_as_float((di + 1) | ((dj + 1) << 2)), x1, y1);
                    queue[2 * e + 1] = make_float4(x2, y2, qv, 0.f);
                } else {
                    zigzag(p, acc, i, j, di, dj, x1, y1, x2, y2, qv);
                }
            }
        }
    }
    __syncthreads();
    const int nq = min(*qn, kQueue);
    if (tid < nq) {
        const float4 r0 = queue[2 * tid], r1 = queue[2 * tid + 1];
        const int c = __float_as_int(r0.x), dd = __float_as_int(r0.y);
        zigzag(p, acc, c >> 16, c & 0xffff, (dd & 3) - 1, ((dd >> 2) & 3) - 1, r0.z, r0.w, r1.x,
               r1.y, r1.z);
    }
}

// Everything one push of one species reads from the host, by value: the
// single-system kernel takes it as its argument, the grouped kernel reads
// each system's from a table in device memory.
struct PushJob {
    P32 p;
    int nub;                             // slot bound known to the host
    const int32_t *nslots;               // slot count on the device
    const uint8_t *kill;
    const float *E[3], *B[3];
    int32_t *cell;
    float *a, *b, *ur, *ut, *up;
    float *J[3];
    unsigned long long *removed;         // this species' removal counters
    uint32_t *err;
    SortPlace SP;                        // placing push: where each slot goes
};

struct PushSmem {
    float *tile, *fld;
    float4 *queue;
    int *box, *qn;
};

// One chunk of kWG * kPPT slots.  Every thread of the workgroup calls it
// and returns from it together.
template <bool SHELL, int kPPT, bool PLACE>
__device__ __forceinline__ void push_block(const PushJob &J, int chunk, const PushSmem &sm) {
    const P32 &p = J.p;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    float *tile = sm.tile, *fld = sm.fld;
    int *box = sm.box;
    // PLACE: the slots before the sort (the slot count already holds the
    // new order's)
    const int n = min(J.nub, J.nslots[PLACE ? 2 : 0]);
    constexpr int kChunk = kWG * kPPT;
    const int base = chunk * kChunk;
    // slots are below 2^30 (the capacity limit), so the byte offset q * 4
    // fits 32 unsigned bits
    const State S{J.cell, J.a, J.b, J.ur, J.ut, J.up};
    const float *Er = J.E[0], *Et = J.E[1], *Ep = J.E[2];
    const float *Br = J.B[0], *Bt = J.B[1], *Bp = J.B[2];
    float *Jr = J.J[0], *Jt = J.J[1], *Jp = J.J[2];

    if (base >= n) return;    // no slot in the chunk (uniform)
    // bounding box of the chunk's cells: every thread loads all its cells at
    // once (a slot past the last reads the last slot's cell and ignores it;
    // behind a branch each, the loads would wait one after the other)
    int imin = 1 << 30, imax = -1, jmin = 1 << 30, jmax = -1;
    int cb[kPPT];
#pragma unroll
    for (int k = 0; k < kPPT; k++) cb[k] = S.ldc((unsigned)min(base + k * kWG + tid, n - 1));
#pragma unroll
    for (int k = 0; k < kPPT; k++) {
        const int q = base + k * kWG + tid;
        const int ck = q < n ? cb[k] : -1;
        if (ck >= 0) {
            const int i = ck >> 16, j = ck & 0xffff;
            imin = min(imin, i); imax = max(imax, i);
            jmin = min(jmin, j); jmax = max(jmax, j);
        }
    }
    if (tid == 0) {
        box[0] = 1 << 30; box[1] = -1; box[2] = 1 << 30; box[3] = -1;
        *sm.qn = 0;
    }
    __syncthreads();
    for (int o = 32; o >= 1; o >>= 1) {
        imin = min(imin, __shfl_xor(imin, o, 64));
        imax = max(imax, __shfl_xor(imax, o, 64));
        jmin = min(jmin, __shfl_xor(jmin, o, 64));
        jmax = max(jmax, __shfl_xor(jmax, o, 64));
    }
    if (lane == 0 && imax >= 0) {
        atomicMin(&box[0], imin); atomicMax(&box[1], imax);
        atomicMin(&box[2], jmin); atomicMax(&box[3], jmax);
    }
    __syncthreads();
    if (box[1] < 0) return;   // no live particle in the chunk (uniform)
    // the patch covers rows [imin-1, imax+2] and columns [jmin-1, jmax+2]:
    // every add of a particle that moves at most one cell lands inside
    const int ti0 = box[0] - 1, tj0 = box[2] - 1;
    const int TI = box[1] - box[0] + 4, TJ = box[3] - box[2] + 4;
    // the field patch: rows [imin-1, imax+1] and columns [jmin-1, jmax+1]
    // within the grid hold every node the chunk's gathers read
    const int fi0 = max(box[0] - 1, 0), fj0 = max(box[2] - 1, 0);
    const int TIf = min(box[1] + 1, p.nr) - fi0 + 1, TJf = min(box[3] + 1, p.nth) - fj0 + 1;
    const bool use_lds = TI * TJ <= kTile && TIf * TJf <= kFld;
    int nkill = 0, nstar = 0, nabs = 0;
    if (use_lds) {
        const int m = TI * TJ;
        for (int e = tid; e < m; e += kWG) {
            tile[e] = 0.f; tile[kTile + e] = 0.f; tile[2 * kTile + e] = 0.f;
        }
        const int mf = TIf * TJf;
        for (int e = tid; e < mf; e += kWG) {
            const int ti = e / TJf, tj = e - ti * TJf;
            const unsigned g = (unsigned)((fi0 + ti) * p.ld + fj0 + tj);
            fld[e * 6 + 0] = ldo(Er, g);
            fld[e * 6 + 1] = ldo(Et, g);
            fld[e * 6 + 2] = ldo(Ep, g);
            fld[e * 6 + 3] = ldo(Br, g);
            fld[e * 6 + 4] = ldo(Bt, g);
            fld[e * 6 + 5] = ldo(Bp, g);
        }
        __syncthreads();
        const Patch P{fld, fi0, fj0, (unsigned)TJf * 24u};
        Acc<true> acc{tile, ti0, tj0, TJ, {Jr, Jt, Jp}, p.ld};
        push_chunk<true, SHELL, kPPT, PLACE>(p, Fields{}, P, acc, n, base, tid, lane, J.kill, S,
                                             J.err, nkill, nstar, nabs, sm.queue, sm.qn, nullptr,
                                             J.SP);
        __syncthreads();
        for (int e = tid; e < m; e += kWG) {
            const int ti = e / TJ, tj = e - ti * TJ;
            const int gi = ti0 + ti, gj = tj0 + tj;
            if (gi < 0 || gi > p.nr || gj < 0 || gj > p.nth) continue;
            const unsigned g = ((unsigned)(gi * p.ld + gj)) << 2;
            const float v0 = tile[e], v1 = tile[kTile + e], v2 = tile[2 * kTile + e];
            if (v0 != 0.f) gadd(reinterpret_cast<float *>(reinterpret_cast<char *>(Jr) + g), v0);
            if (v1 != 0.f) gadd(reinterpret_cast<float *>(reinterpret_cast<char *>(Jt) + g), v1);
            if (v2 != 0.f) gadd(reinterpret_cast<float *>(reinterpret_cast<char *>(Jp) + g), v2);
        }
    } else {
        // the gather reads the fields through buffer resources in this mode
        // (nr + 1) * ld stays near the 2^29-node grid limit, so the byte count
        // fits 32 unsigned bits
        const int nbytes = (int)((unsigned)(p.nr + 1) * (unsigned)p.ld * 4u);
        Fields F;
        F.er = __builtin_amdgcn_make_buffer_rsrc((void *)Er, 0, nbytes, kRsrcWord3);
        F.et = __builtin_amdgcn_make_buffer_rsrc((void *)Et, 0, nbytes, kRsrcWord3);
        F.ep = __builtin_amdgcn_make_buffer_rsrc((void *)Ep, 0, nbytes, kRsrcWord3);
        F.br = __builtin_amdgcn_make_buffer_rsrc((void *)Br, 0, nbytes, kRsrcWord3);
        F.bt = __builtin_amdgcn_make_buffer_rsrc((void *)Bt, 0, nbytes, kRsrcWord3);
        F.bp = __builtin_amdgcn_make_buffer_rsrc((void *)Bp, 0, nbytes, kRsrcWord3);
        Acc<false> acc{nullptr, 0, 0, 0, {Jr, Jt, Jp}, p.ld};
        const int kc = lane_comp(lane);
        float *kg = kc == 0 ? Jr : (kc == 1 ? Jt : Jp);
        push_chunk<false, SHELL, kPPT, PLACE>(p, F, Patch{nullptr, 0, 0, 0u}, acc, n, base, tid,
                                              lane, J.kill, S, J.err, nkill, nstar, nabs,
                                              sm.queue, sm.qn, kg, J.SP);
    }
    int tk = nkill, ts = nstar, ta = nabs;
    for (int o = 32; o >= 1; o >>= 1) {
        tk += __shfl_xor(tk, o, 64);
        ts += __shfl_xor(ts, o, 64);
        ta += __shfl_xor(ta, o, 64);
    }
    if (lane == 0) {
        if (tk) atomicAdd(&J.removed[1], (unsigned long long)tk);
        if (ts) atomicAdd(&J.removed[2], (unsigned long long)ts);
        if (ta) atomicAdd(&J.removed[3], (unsigned long long)ta);
    }
}

// six waves per SIMD: the prefetched momentum fits in 80 VGPRs without spills
template <bool SHELL, int kPPT, bool PLACE>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_push32(const PushJob J) {
    __shared__ float tile[3 * kTile];
    __shared__ float fld[6 * kFld];
    __shared__ float4 queue[2 * kQueue];
    __shared__ int box[4];
    __shared__ int qn;
    push_block<SHELL, kPPT, PLACE>(J, (int)blockIdx.x, PushSmem{tile, fld, queue, box, &qn});
}

// The pushes of many systems in one launch of persistent workgroups: each
// workgroup takes chunks (items) from a counter in device memory until none
// is left.  Job k owns items [starts[k], starts[k + 1]).  The workgroup that
// finishes last returns both counters to zero for the next launch.
template <bool SHELL, int kPPT, bool PLACE>
__global__ void __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_push32_group(const PushJob *__restrict__ jobs, const int *__restrict__ starts, int njobs,
               int *__restrict__ ctr) {
    __shared__ float tile[3 * kTile];
    __shared__ float fld[6 * kFld];
    __shared__ float4 queue[2 * kQueue];
    __shared__ int box[4];
    __shared__ int qn;
    __shared__ int next, job;
    __shared__ uint32_t stage[kJobWords];
    const PushSmem sm{tile, fld, queue, box, &qn};
    const int total = starts[njobs];
    if (threadIdx.x == 0) next = atomicAdd(&ctr[0], 1);
    __syncthreads();
    int item = __builtin_amdgcn_readfirstlane(next);
    while (item < total) {
        find_job(starts, njobs, item, &job);
        // the next item is taken now, so that the counter's round trip
        // overlaps this item's work
        int nx = 0;
        if (threadIdx.x == 0) nx = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int lo = __builtin_amdgcn_readfirstlane(job);
        // a plain push reads no placement pointers (the job's last member)
        const PushJob J =
            stage_uniform(jobs + lo, stage, PLACE ? sizeof(PushJob) : offsetof(PushJob, SP));
        push_block<SHELL, kPPT, PLACE>(J, item - starts[lo], sm);
        if (threadIdx.x == 0) next = nx;
        __syncthreads();
        item = __builtin_amdgcn_readfirstlane(next);
    }
    group_done(ctr);
}

// the kernel instance of a species' push: particles per thread, shell,
// placing
struct PushKey {
    int ppt;
    bool shell, place;
};

// ppt: particles per thread, 0 = the context's own setting
PushKey push_key(const ffpic_ctx *c, int s, int ppt = 0) {
    const int v = ppt > 0 ? ppt : c->push_ppt;
    return {v == 8 || v == 32 ? v : 16, c->d.shell_r > c->d.rmin, c->sort_pending[s]};
}

int push_key_index(const PushKey &k) {
    return (k.ppt == 8 ? 0 : (k.ppt == 16 ? 1 : 2)) + (k.shell ? 3 : 0) + (k.place ? 6 : 0);
}

// the job of one species' push from the context's state, and the host
// bookkeeping that follows the launch (a placing push leaves the new order
// in the second buffer)
PushJob make_push_job(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    PushJob J{};
    P32 &p = J.p;
    p.nr = c->nr; p.nth = c->nth; p.ld = c->ld;
    p.dlog = (float)c->dlog; p.dth = (float)c->dth; p.dt = (float)c->dt;
    p.inv_dlog = (float)(1.0 / c->dlog);
    p.inv_dth = (float)(1.0 / c->dth);
    double xa = log(c->d.r_abs / c->d.rmin) / c->dlog;
    p.iabs = (int)floor(xa);
    p.aabs = (float)(xa - floor(xa));
    p.rn = (const float *)c->dtab[T_RN];
    p.sn = (const float *)c->dtab[T_SN];
    p.cn = (const float *)c->dtab[T_CN];
    double qm = S.qm;
    p.Q = (float)((qm > 0 ? 1.0 : -1.0) * S.weight);
    p.h = (float)(0.5 * c->dt * c->d.omega_b * qm);
    p.kk = (float)(c->dt * c->d.rr_coef * rr_factor(c) * fabs(qm) * fabs(qm) * fabs(qm));
    // the shell radius in cell units, split like r_abs
    const bool shell = c->d.shell_r > c->d.rmin;
    const double xs = shell ? log(c->d.shell_r / c->d.rmin) / c->dlog : 0.0;
    p.ishell = (int)floor(xs);
    p.ashell = (float)(xs - floor(xs));
    J.nub = (int)S.nub;
    const bool place = c->sort_pending[s];
    // the placing push runs over the slots before the sort: the third
    // entry of the sort's totals
    J.nslots = place ? (const int32_t *)c->sort_tot[s] : c->nslots + s;
    J.kill = c->kill;
    for (int k = 0; k < 3; k++) {
        J.E[k] = (const float *)c->E[k];
        J.B[k] = (const float *)c->B[k];
        J.J[k] = (float *)c->J[k];
    }
    J.cell = (int32_t *)S.cur[0];
    J.a = (float *)S.cur[1];
    J.b = (float *)S.cur[2];
    J.ur = (float *)S.cur[3];
    J.ut = (float *)S.cur[4];
    J.up = (float *)S.cur[5];
    J.removed = c->removed + 4 * s;
    J.err = c->err;
    if (place) J.SP = c->place[s];
    return J;
}

void after_push(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    if (c->sort_pending[s]) {
        for (int a = 0; a < S.narr; a++) std::swap(S.cur[a], S.alt[a]);
        c->sort_pending[s] = false;
    }
}

using PushKern = void (*)(const PushJob);
using PushGroupKern = void (*)(const PushJob *, const int *, int, int *);

template <bool SHELL, bool PLACE>
PushKern push_kern(int ppt) {
    return ppt == 8 ? k_push32<SHELL, 8, PLACE>
                    : (ppt == 32 ? k_push32<SHELL, 32, PLACE> : k_push32<SHELL, 16, PLACE>);
}
template <bool SHELL, bool PLACE>
PushGroupKern push_group_kern(int ppt) {
    return ppt == 8 ? k_push32_group<SHELL, 8, PLACE>
                    : (ppt == 32 ? k_push32_group<SHELL, 32, PLACE>
                                 : k_push32_group<SHELL, 16, PLACE>);
}

void push32(ffpic_ctx *c, int s) {
    ffpic::Species &S = c->sp[s];
    if (S.nub == 0) return;
    const PushKey k = push_key(c, s);
    const PushJob J = make_push_job(c, s);
    const int chunk = kWG * k.ppt;
    const int nb = (int)((S.nub + chunk - 1) / chunk);
    const PushKern kern = k.shell ? (k.place ? push_kern<true, true>(k.ppt) : push_kern<true, false>(k.ppt))
                                  : (k.place ? push_kern<false, true>(k.ppt) : push_kern<false, false>(k.ppt));
    hipLaunchKernelGGL(kern, dim3(nb), dim3(kWG), 0, c->stream, J);
    FFPIC_LAUNCH_CHECK();
    after_push(c, s);
}

// ---- grouped pushes of several contexts (batches)

size_t push_job_bytes() { return sizeof(PushJob); }

int push_group_key(const ffpic_ctx *c, int s, int ppt) {
    return push_key_index(push_key(c, s, ppt));
}

int push_job(ffpic_ctx *c, int s, void *out, int ppt) {
    ffpic::Species &S = c->sp[s];
    const PushKey k = push_key(c, s, ppt);
    const PushJob J = make_push_job(c, s);
    std::memcpy(out, &J, sizeof(J));
    after_push(c, s);
    const int chunk = kWG * k.ppt;
    return (int)((S.nub + chunk - 1) / chunk);
}

static PushGroupKern group_kern_of(int key) {
    const int ppt = key % 3 == 0 ? 8 : (key % 3 == 1 ? 16 : 32);
    const bool shell = (key / 3) % 2 != 0, place = key >= 6;
    return shell ? (place ? push_group_kern<true, true>(ppt) : push_group_kern<true, false>(ppt))
                 : (place ? push_group_kern<false, true>(ppt) : push_group_kern<false, false>(ppt));
}

int push_group_slots(int key) {
    int per_cu = 0, cus = 0, dev = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)group_kern_of(key), kWG,
                                                     0) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 1024;
    }
    return std::max(1, per_cu) * std::max(1, cus);
}

void push_group_launch(hipStream_t st, int key, const void *jobs, const int *starts, int njobs,
                       int grid, int *ctr) {
    hipLaunchKernelGGL(group_kern_of(key), dim3(grid), dim3(kWG), 0, st,
                       (const PushJob *)jobs, starts, njobs, ctr);
    FFPIC_LAUNCH_CHECK();
}

}  // namespace ffpic
