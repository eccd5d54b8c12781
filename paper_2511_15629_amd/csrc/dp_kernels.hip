// HIP kernels for gfx950 (CDNA4): per-stage expectation on MFMA, max-plus Bellman sweep
// with argmax on the VALU, and the adjoint stage kernels.
//
// Method: backward induction of Eq. (5)-(6) in the tensor form of Algorithm 1, with the
// expectation generalised to a Markov chain (W_t = P_t V_{t+1}) and the action axis
// restricted to whole grid steps (the recombining grid of Sec. III-A).
#include "dp_internal.h"

#include <math.h>

namespace dpk {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------------------------
// Payoff of a move of d grid steps (Eq. (1) objective with the transition of Eq. (2)):
// g(d) MWh sold to the grid, r = lam g - c_deg |g| - c_start [d != 0].
// ------------------------------------------------------------------------------------
__device__ __forceinline__ float move_energy(int d, const Payoff &p)
{
    float fd = (float)d;
    if (d > 0) return -(fd * p.delta) / p.eta_c;
    if (d < 0) return -(fd * p.delta) * p.eta_d;
    return 0.0f;
}

// Price-independent part of the payoff: h(d) = -c_deg |g(d)| - c_start [d != 0].
__device__ __forceinline__ float move_cost(int d, const Payoff &p)
{
    const float h = -(p.c_deg * fabsf(move_energy(d, p)));
    return d != 0 ? h - p.c_start : h;
}

// r(lam, d) = lam g(d) + h(d), one fused multiply-add (the same rounding in every kernel).
__device__ __forceinline__ float move_reward(float lam, int d, const Payoff &p)
{
    return fmaf(lam, move_energy(d, p), move_cost(d, p));
}

// ------------------------------------------------------------------------------------
// Expectation C = A * B on MFMA (v_mfma_f32_16x16x4_f32, FP32 products and accumulation).
// A is K x K (P_t, or its transpose), B is K x N with leading dimension ldb, C is K x N.
// The tile chain: a 16 x 16 tile (tm, tn) of C is accumulated from zero over the k-steps
// st = 0 .. ceil(K/4) - 1 in ascending order, one MFMA per step on A[16 tm + i][4 st + kk]
// and B[4 st + kk][16 tn + j] (zero outside the matrices).  Every expectation kernel (the
// single solve, the adjoint's transport, the batch's panels and strips) runs exactly this
// chain per tile, so their results are bitwise equal.  The operand loads of a chunk of CH
// steps are all issued before its MFMAs, so a chunk costs one memory round trip.
// Lane layout of the 16x16x4 instruction: A[i][kk] from lane i + 16 kk, B[kk][j] from
// lane j + 16 kk, result row 4 (lane / 16) + v, column lane % 16 in register v.
// ------------------------------------------------------------------------------------
// Strip of NT adjacent 16 x 16 tiles (16 rows x 16 NT columns) per wave: each step loads
// one A operand and NT B operands and issues NT MFMAs, so A loads and per-wave setup are
// shared by NT tiles.  Each tile runs the tile chain (operands, order), so the results
// are bitwise those of the other expectation kernels.
template <int CH, int NT>
__device__ __forceinline__ void contract_strip(const float *__restrict__ A,
                                               const float *__restrict__ B, int ldb,
                                               float *__restrict__ C, int ldc, int K, int N,
                                               int tm, int tn0)
{
    const int lane = threadIdx.x & 63;
    const int arow = tm * 16 + (lane & 15);
    const int kq = lane >> 4;
    const bool rok = arow < K;
    int col[NT];
    bool cok[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        col[n] = (tn0 + n) * 16 + (lane & 15);
        cok[n] = col[n] < N;
    }
    floatx4 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4 * CH) {
        float av[CH], bv[CH][NT];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int kx = k0 + 4 * i + kq;
            const bool kok = kx < K;
            av[i] = (kok && rok) ? A[(size_t)arow * K + kx] : 0.f;
#pragma unroll
            for (int n = 0; n < NT; ++n)
                bv[i][n] = (kok && cok[n]) ? B[(size_t)kx * ldb + col[n]] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (k0 + 4 * i < K) {
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i][n], acc[n], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        if (cok[n]) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = tm * 16 + 4 * kq + v;
                if (r < K) C[(size_t)r * ldc + col[n]] = acc[n][v];
            }
        }
    }
}

// P_t in the lane order of the 16x16x4 instruction: for row tile tm and k-step st, the 64
// A operands A[16 tm + i][4 st + kk] (lane i + 16 kk) are 64 consecutive floats, zero
// outside the K x K matrix.  Each A load of the tile is then one coalesced 256-byte read
// instead of 16 rows' 16-byte pieces.  Layout per stage: [ceil(K/16)][ceil(K/4)][64].
size_t packed_P_floats(int K) { return (size_t)((K + 15) >> 4) * ((K + 3) >> 2) * 64; }

// TRANS: pack P_t^T instead (A[r][c] = P_t[c][r]), for the adjoint's transport.
template <bool TRANS>
__global__ void pack_P_kernel(const float *__restrict__ P, int K, int nstage,
                              float *__restrict__ Pp)
{
    const int ntm = (K + 15) >> 4, nst = (K + 3) >> 2;
    const size_t per = (size_t)ntm * nst * 64, n = per * nstage;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t t = e / per, r = e - t * per;
        const int l = (int)(r & 63), st = (int)((r >> 6) % nst), tm = (int)((r >> 6) / nst);
        const int row = tm * 16 + (l & 15), col = 4 * st + (l >> 4);
        const size_t src = TRANS ? (size_t)col * K + row : (size_t)row * K + col;
        Pp[e] = (row < K && col < K) ? P[t * K * K + src] : 0.f;
    }
}

hipError_t launch_pack_P(const float *P, bool transA, int K, int nstage, float *Pp,
                         hipStream_t stream)
{
    const size_t n = packed_P_floats(K) * nstage;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (transA)
        hipLaunchKernelGGL(pack_P_kernel<true>, dim3(blocks), dim3(256), 0, stream, P, K, nstage, Pp);
    else
        hipLaunchKernelGGL(pack_P_kernel<false>, dim3(blocks), dim3(256), 0, stream, P, K, nstage, Pp);
    return hipGetLastError();
}

// The tile chain with A read from the packed layout (A = P_t, or P_t^T when packed
// transposed); CH = 32 loads every operand of a tile up to K = 128 in one round trip.
template <int CH = 32>
__device__ __forceinline__ void contract_tile_packed(const float *__restrict__ Ap,
                                                     const float *__restrict__ B, int ldb,
                                                     float *__restrict__ C, int ldc, int K,
                                                     int N, int tm, int tn)
{
    const int lane = threadIdx.x & 63;
    const int kq = lane >> 4;
    const int col = tn * 16 + (lane & 15);
    const bool cok = col < N;
    const int nst = (K + 3) >> 2;
    const float *ap = Ap + (size_t)tm * nst * 64 + lane;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4 * CH) {
        float av[CH], bv[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int st = (k0 >> 2) + i;
            const int kx = 4 * st + kq;
            av[i] = st < nst ? ap[(size_t)st * 64] : 0.f;
            bv[i] = (kx < K && cok) ? B[(size_t)kx * ldb + col] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            if (k0 + 4 * i < K) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i], acc, 0, 0, 0);
        }
    }
    if (cok) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = tm * 16 + 4 * kq + v;
            if (r < K) C[(size_t)r * ldc + col] = acc[v];
        }
    }
}

__global__ __launch_bounds__(256) void contract_packed_kernel(const float *__restrict__ Ap,
                                                              const float *__restrict__ B,
                                                              int ldb, float *__restrict__ C,
                                                              int ldc, int K, int N)
{
    const int ntm = (K + 15) >> 4;
    const int ntn = (N + 15) >> 4;
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= ntm * ntn) return;
    contract_tile_packed(Ap, B, ldb, C, ldc, K, N, wid % ntm, wid / ntm);
}

hipError_t launch_contract_packed(const float *Ap, const float *B, int ldb, float *C, int ldc,
                                  int K, int N, hipStream_t stream)
{
    const int tiles = ((K + 15) / 16) * ((N + 15) / 16);
    const int blocks = (tiles + 3) / 4;
    hipLaunchKernelGGL(contract_packed_kernel, dim3(blocks), dim3(256), 0, stream, Ap, B, ldb,
                       C, ldc, K, N);
    return hipGetLastError();
}


// ------------------------------------------------------------------------------------
// Max-plus Bellman sweep with argmax (Eq. (5); Algorithm 1's gather, -inf mask, payoff and
// maximum over the action axis), evaluated as exact sliding-window maxima.
//
// The payoff of a move of d grid steps is affine in d on each side of the idle move
// (Eq. (1) with the transition of Eq. (2)): r(d) = A_c d - c_start for d > 0 with
// A_c = -(lam + c_deg) delta / eta_c, and r(d) = A_d d - c_start for d < 0 with
// A_d = -(lam - c_deg) delta eta_d.  So for output s the charge candidates
// W[j] + r(j - s), j = s + 1 .. s + w_up, are u_c[j] - A_c s - c_start with
// u_c[j] = W[j] + A_c j: the best of them is the maximum of u_c over a window of w_up
// consecutive next states, the same window shape for every s.  The discharge side is the
// window j = s - w_down .. s - 1 of u_d[j] = W[j] + A_d j, and the idle move is W[s].
// Next states outside [0, S) carry W = -inf (the infeasibility mask).
//
// Maxima over windows of a fixed width w (van Herk; Gil and Werman): cut the next-state
// axis into segments of w.  A window starting at e covers the end of e's segment and the
// start of the next one, so its maximum is the larger of the suffix maximum of e's
// segment from e and the prefix maximum of the next segment up to e + w - 1.  Prefix and
// suffix maxima are segmented scans: a lane scans a run of 8 next states, the runs of a
// wave are joined by a segmented shuffle scan, and consecutive passes of a wave by a carry.
// Each output then reads two table entries per side instead of w candidates.
//
// Decisions.  u is formed in FP32 by one fma at the absolute next state j, so every output
// ranks the same u values whatever tile it belongs to: results do not depend on the tiling
// or on the launch.  Within a side the smallest next state attaining the maximum of u is
// taken (prefix scans keep the earlier entry on ties, suffix scans the later-scanned,
// smaller one, and a window's suffix part wins over its prefix part).  The side's
// candidate is then re-evaluated in FP64 as W[j] + r(j - s), and the sides are compared in
// next-state order -- discharge (j < s), idle (j = s), charge (j > s) -- each later one
// only when strictly larger.  The value is rounded to FP32 once, from that FP64 candidate.
// Ranking by the rounded u can prefer a candidate within the rounding of |W| + |A j| of
// the exact maximum (a near-tie); the value carried on is that candidate's own.
//
// Block = one price state k and a tile of TS consecutive SoC indices, on NW waves.
// ------------------------------------------------------------------------------------
// Sum of the K entries of a row of P_t in FP64, the same in every wave and every kernel:
// lane l adds entries l, l + 64, ... in ascending order, then a xor butterfly (each step
// adds the same two operands on both lanes, so every lane ends with the same bits).
__device__ __forceinline__ double row_sum_f64(const float *__restrict__ row, int K, int lane)
{
    double acc = 0.0;
    for (int c = lane; c < K; c += 64) acc += (double)row[c];
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) acc += __shfl_xor(acc, m);
    return acc;
}

// Barrier between a tile's LDS phases: the block's, or for a one-wave tile only a code
// motion fence (one wave's LDS operations complete in program order).
template <int NW>
__device__ __forceinline__ void sweep_sync()
{
    if constexpr (NW == 1)
        __builtin_amdgcn_wave_barrier();
    else
        __syncthreads();
}

// A candidate of the window scans: its u value and its position e in the side's array
// (value -inf: none).
struct Cand {
    float v;
    int e;
};

// The better of a (earlier in scan order) and b; TIE_A: a tie keeps a.
template <bool TIE_A>
__device__ __forceinline__ Cand better(const Cand &a, const Cand &b)
{
    const bool keep_a = TIE_A ? (a.v >= b.v) : (a.v > b.v);
    return keep_a ? a : b;
}

// Payoff slopes of Eq. (1) per grid step on the charge and discharge sides, FP64.
__device__ __forceinline__ double slope_charge(float lam, const Payoff &p)
{
    return -((double)lam + (double)p.c_deg) * (double)p.delta / (double)p.eta_c;
}
__device__ __forceinline__ double slope_discharge(float lam, const Payoff &p)
{
    return -((double)lam - (double)p.c_deg) * (double)p.delta * (double)p.eta_d;
}

// Layout of a side with w moves over a tile of TS outputs (n = TS + w - 1 entries): the u
// array, -inf from n up to un = n rounded up to 8 (the scans' range); then the prefix
// table g, indexed by e - glo(w) over TS + 16 entries (glo: w - 1 rounded down to 8), and
// the suffix table h, indexed by e over the same count.  A table entry is the position of
// the maximum (16 bits: positions stay below 2^15); its value is u at that position.
__host__ __device__ __forceinline__ int scan_un(int TS, int w) { return (TS + w - 1 + 7) & ~7; }
__host__ __device__ __forceinline__ int scan_glo(int w) { return (w - 1) & ~7; }
__host__ __device__ __forceinline__ int scan_tab_words(int TS) { return (TS + 16) / 2; }

// The candidate a table entry names: u at position p.  A window whose entries are all -inf
// may carry no position (stored as 0xffff), which reads as -inf.
__device__ __forceinline__ Cand table_cand(const float *u, int un, int p)
{
    const float v = u[min(p, un - 1)];
    return Cand{p < un ? v : -INFINITY, p};
}

// Short move ranges take the direct maximum over the whole range (an add and half a
// v_max3 per candidate, on chunks of DIRECT_D moves for DIRECT_R outputs per lane); longer
// ones the window scans of the hoisted payoff, whose cost per output does not grow with the
// range.
constexpr int DIRECT_SPAN = 96, DIRECT_R = 4, DIRECT_D = 8;
__host__ __device__ __forceinline__ bool sweep_direct(int w_up, int w_down)
{
    return w_up + w_down + 1 <= DIRECT_SPAN;
}

// Words of a side's LDS (0 for a side without moves); a multiple of 8.
__host__ __device__ __forceinline__ int side_words(int TS, int w)
{
    if (w == 0) return 0;
    return scan_un(TS, w) + 2 * scan_tab_words(TS);
}

// Scan-order absorption of candidate (v, e) into acc: a segment boundary (head) starts
// anew; otherwise acc keeps its candidate unless v is larger (FWD: acc holds the smaller
// positions, ties keep it) or at least as large (backward: v has the smaller position).
// Written as one predicate and two selects.
template <bool FWD>
__device__ __forceinline__ void absorb(Cand &acc, float v, int e, bool head)
{
    const bool take = head | (FWD ? v > acc.v : v >= acc.v);
    acc.v = take ? v : acc.v;
    acc.e = take ? e : acc.e;
}

// One step of a segmented inclusive scan across the wave's lanes: lane l takes the
// candidate of the lane the DPP control names (unless a segment boundary already lies in
// the lanes it covers), and the boundary flags are or-ed.  Lanes without a source lane,
// or outside the row mask, see (-inf, -1, no boundary).
template <bool FWD, int CTRL, int ROWS>
__device__ __forceinline__ void dpp_scan_step(Cand &acc, int &flag)
{
    const float ov = __int_as_float(__builtin_amdgcn_update_dpp(
        (int)0xff800000, __float_as_int(acc.v), CTRL, ROWS, 0xf, false));
    const int oe = __builtin_amdgcn_update_dpp(-1, acc.e, CTRL, ROWS, 0xf, false);
    const int of = __builtin_amdgcn_update_dpp(0, flag, CTRL, ROWS, 0xf, false);
    // the other lane's candidate is earlier in scan order: it wins ties forward
    const bool take = !flag & (FWD ? ov >= acc.v : ov > acc.v);
    acc.v = take ? ov : acc.v;
    acc.e = take ? oe : acc.e;
    flag |= of;
}

// One wave's segmented max-scan of u[e] over e in [r0, r1) (both multiples of 8), whose
// segments are [phi + m w, phi + (m + 1) w) cut to the range (the range starts and ends
// segments).  FWD: the positions of the prefix maxima g(e) over [segment start, e],
// written at tg[e - glo] for runs inside [glo, glo + TS + 16); otherwise those of the
// suffix maxima h(e) over [e, segment end], written at tg[e] for runs inside [0, TS); a
// run's 8 positions go out as one 16-byte store.
// Lane l of a pass holds the run of 8 entries t = p0 + 8 l .. p0 + 8 l + 7 in scan order
// (e = r0 + t forward, r1 - 1 - t backward).  A first pass over the run gives the lane's
// total; DPP row shifts within rows of 16 lanes and row broadcasts of lanes 15 and 31
// join the lanes' totals; a second pass rescans the run from the lane's exclusive prefix.
template <bool FWD>
__device__ __forceinline__ void window_scan(const float *__restrict__ u, int un, int w, int phi,
                                            int r0, int r1, int glo, int TS,
                                            uint16_t *__restrict__ tg, int lane)
{
    const Cand none = {-INFINITY, -1};
    const int len = r1 - r0;
    Cand carry = none;                         // inclusive result at the previous pass's end
    for (int p0 = 0; p0 < len; p0 += 512) {
        const int t0 = p0 + 8 * lane;
        // the run's entries (its first entry e0; lanes past the range read in-bounds data
        // and come after every lane of the range in scan order)
        const int e0 = FWD ? r0 + t0 : r1 - 1 - t0;
        float x[8];
        {
            const int lo = FWD ? min(e0, un - 8) : max(e0, 7) - 7;
            const float4 a4 = *reinterpret_cast<const float4 *>(u + lo);
            const float4 b4 = *reinterpret_cast<const float4 *>(u + lo + 4);
            const float y[8] = {a4.x, a4.y, a4.z, a4.w, b4.x, b4.y, b4.z, b4.w};
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = y[FWD ? q : 7 - q];
        }
        // segment boundaries in the run: bit q when entry q starts a segment in scan order
        int mask = t0 == 0 ? 1 : 0;
        {
            const int dm = FWD ? e0 - phi : phi - 1 - e0;      // entry q: dm + q = 0 mod w
            int r = dm % w;
            r = r < 0 ? r + w : r;
            if (w >= 8) {                              // at most one boundary in the run
                const int q1 = r == 0 ? 0 : w - r;
                mask |= q1 < 8 ? 1 << q1 : 0;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    mask |= (r == 0) << q;
                    r = r + 1 == w ? 0 : r + 1;
                }
            }
        }
        Cand acc = lane == 0 ? carry : none;
#pragma unroll
        for (int q = 0; q < 8; ++q) absorb<FWD>(acc, x[q], FWD ? e0 + q : e0 - q, (mask >> q) & 1);
        int flag = mask != 0;
        dpp_scan_step<FWD, 0x111, 0xf>(acc, flag);     // row_shr:1
        dpp_scan_step<FWD, 0x112, 0xf>(acc, flag);     // row_shr:2
        dpp_scan_step<FWD, 0x114, 0xf>(acc, flag);     // row_shr:4
        dpp_scan_step<FWD, 0x118, 0xf>(acc, flag);     // row_shr:8
        dpp_scan_step<FWD, 0x142, 0xa>(acc, flag);     // row_bcast:15 into rows 1, 3
        dpp_scan_step<FWD, 0x143, 0xc>(acc, flag);     // row_bcast:31 into rows 2, 3
        // the lane's exclusive prefix (wave_shr:1); lane 0 continues the previous pass
        Cand run = {__int_as_float(__builtin_amdgcn_update_dpp(
                        (int)0xff800000, __float_as_int(acc.v), 0x138, 0xf, 0xf, false)),
                    __builtin_amdgcn_update_dpp(-1, acc.e, 0x138, 0xf, 0xf, false)};
        if (lane == 0) run = carry;
        carry = Cand{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(acc.v), 63)),
                     __builtin_amdgcn_readlane(acc.e, 63)};
        // runs lie wholly inside or outside the written ranges (all bounds are multiples
        // of 8)
        const int i0 = FWD ? e0 - glo : e0 - 7;
        if (t0 < len && i0 >= 0 && i0 < (FWD ? TS + 16 : TS)) {
            unsigned pos[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                absorb<FWD>(run, x[q], FWD ? e0 + q : e0 - q, (mask >> q) & 1);
                pos[FWD ? q : 7 - q] = (unsigned)run.e & 0xffffu;
            }
            *reinterpret_cast<uint4 *>(tg + i0) =
                make_uint4(pos[0] | pos[1] << 16, pos[2] | pos[3] << 16, pos[4] | pos[5] << 16,
                           pos[6] | pos[7] << 16);
        }
    }
}

// smem: this tile's LDS (sweep_lds_bytes); tid: thread index within the tile's NW waves.
// LDS: per side (discharge, then charge) the u array and the g and h tables; the
// expectation row over next states s0 - w_down .. s0 + TS - 1 + w_up; with the fused
// expectation, row k of P_t.
// DIRECT: the block's move range takes the direct maximum (sweep_direct(w_up, w_down)).
// RB: rows of V_{t+1} per load batch of the fused expectation (fused_rows(K)).
template <int NW, bool DIRECT, int RB = 8>
__device__ __forceinline__ void sweep_block(const SweepArgs &a, const int k, const int tile,
                                            const int TS, float *smem, const int tid)
{
    const int s0 = tile * TS;
    const int S = a.S, w_up = a.w_up, w_down = a.w_down;
    const int jlo = s0 - w_down;                        // Wl[i] holds next state jlo + i
    const int nwl = TS + w_down + w_up;
    // direct mode: the W row (-inf up to wl_alloc) and the reward row over nchunk chunks;
    // scan mode: both sides' u arrays and tables, then the W row
    constexpr bool direct = DIRECT;
    const int span = w_up + w_down + 1;
    const int nchunk = (span + DIRECT_D - 1) / DIRECT_D;
    const int wl_alloc = (TS + span + DIRECT_D + 3) & ~3;
    const int wd_words = direct ? 0 : side_words(TS, w_down), tb = scan_tab_words(TS);
    float *const side_d = smem, *const side_c = smem + wd_words;   // discharge, charge
    float *Wl = smem + wd_words + (direct ? 0 : side_words(TS, w_up));
    float *rl = Wl + wl_alloc;                          // direct mode: reward row

    const float NEG = -INFINITY;
    float lam = 0.0f, shift = 0.0f;
    double off_next = 0.0, rsum_m1 = 0.0;
    // u arrays of both sides, formed as the expectation row is written: discharge
    // e = 0 .. TS + w_down - 2 at next state s0 - w_down + e (Wl[e]); charge
    // e = 0 .. TS + w_up - 2 at next state s0 + 1 + e (Wl[w_down + 1 + e]); -inf up to the
    // arrays' rounded length.  Output o's window is e = o .. o + w - 1 on either side.
    float Ad = 0.0f, Ac = 0.0f;                         // FP32 slopes (lam known first)
    const int nd = (w_down && !direct) ? TS + w_down - 1 : 0;
    const int nc = (w_up && !direct) ? TS + w_up - 1 : 0;
    auto put = [&](int i, float v) {                    // next state jlo + i, value v
        Wl[i] = v;
        const float jf = (float)(jlo + i);
        if (i < nd) side_d[i] = fmaf(Ad, jf, v);
        const int ec = i - w_down - 1;
        if (ec >= 0 && ec < nc) side_c[ec] = fmaf(Ac, jf, v);
    };
    if constexpr (direct) {
        for (int i = nwl + tid; i < wl_alloc; i += NW * 64) Wl[i] = NEG;
    } else {
        const int ud = w_down ? scan_un(TS, w_down) : 0, uc = w_up ? scan_un(TS, w_up) : 0;
        for (int e = nd + tid; e < ud; e += NW * 64) side_d[e] = NEG;
        for (int e = nc + tid; e < uc; e += NW * 64) side_c[e] = NEG;
    }
    if (a.Vn) {
        // Fused expectation (the single solve): the block forms the row it needs,
        // W_t[k][j] = sum_k' P_t[k][k'] V_{t+1}[k'][j] over the staged next states, from the
        // normalised V_{t+1} and row k of P_t.  Each entry is an FP32 fma chain over k'
        // ascending from 0 (zero terms past K add exact zeros): bitwise the MFMA tile chain of
        // the expectation kernels, which pads to a multiple of 4.  A thread owns quads of four
        // next states (one 16-byte load per row), with the next RB rows' loads in flight while
        // RB are accumulated.
        lam = a.lam[k];
        shift = a.Vn[0];                           // the stage's normalisation V_{t+1}[0][0]
        off_next = a.off_next[0];
        rsum_m1 = a.rho1 ? a.rho1[k] : 0.0;
        Ad = (float)slope_discharge(lam, a.pay);
        Ac = (float)slope_charge(lam, a.pay);
        const int K = a.K;
        const float *Pk = a.P + (size_t)k * K;
        // Row k of P_t goes to LDS (zero-padded to a multiple of RB), its loads issued before
        // the first rows of V_{t+1}, and is read back as broadcasts.  Rows past K enter with
        // P = 0 and the last row's values, adding exact zeros (the chain's sums are never
        // -0), as the tile chain's padding does; quads outside [0, S) read row data at
        // state 0 and are replaced by -inf.  RB (8 or 10, whichever pads K less) sets how
        // many of those repeated loads there are: none for K = 20, 50, 100 with 10.
        static_assert(RB % 2 == 0, "P is read back in pairs");
        const int K8 = (K + RB - 1) / RB * RB;
        float *prow = direct ? rl + nchunk * DIRECT_D : Wl + ((nwl + 3) & ~3);   // [K8]
        const int q0 = jlo >> 2;                   // quads of next states (floor: jlo < 0 ok)
        const int q1 = (jlo + nwl + 3) >> 2;
        float pmine[4];                            // this thread's first P entries
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = tid + u * NW * 64;
            pmine[u] = i < K ? Pk[i] : 0.0f;
        }
        auto load = [&](float4 (&v)[RB], const float *vq, int r0) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int kc = min(r0 + r, K - 1);
                v[r] = *reinterpret_cast<const float4 *>(vq + (size_t)kc * a.ldvn);
            }
        };
        float4 va[RB], vb[RB];
        {
            const int j0 = 4 * (q0 + tid);
            load(va, a.Vn + ((j0 >= 0 && j0 < S) ? j0 : 0), 0);    // first quad's first rows
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = tid + u * NW * 64;
            if (i < K8) prow[i] = pmine[u];
        }
        for (int i = tid + 4 * NW * 64; i < K8; i += NW * 64)   // rows beyond 4 per thread
            prow[i] = i < K ? Pk[i] : 0.0f;
        sweep_sync<NW>();
        for (int q = q0 + tid; q < q1; q += NW * 64) {
            const int j0 = 4 * q;
            const bool in = j0 >= 0 && j0 < S;     // j0 < S <= ldvn: the quad is in the row
            const float *vq = a.Vn + (in ? j0 : 0);
            if (q != q0 + tid) load(va, vq, 0);
            float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            auto accumulate = [&](const float4 (&v)[RB], int r0) {
                const float2 *p2 = reinterpret_cast<const float2 *>(prow + r0);
#pragma unroll
                for (int r2 = 0; r2 < RB / 2; ++r2) {
                    const float2 pp = p2[r2];
                    const float pr[2] = {pp.x, pp.y};
#pragma unroll
                    for (int r = 0; r < 2; ++r) {
                        const float4 x = v[2 * r2 + r];
                        acc.x = fmaf(pr[r], x.x, acc.x);
                        acc.y = fmaf(pr[r], x.y, acc.y);
                        acc.z = fmaf(pr[r], x.z, acc.z);
                        acc.w = fmaf(pr[r], x.w, acc.w);
                    }
                }
            };
            for (int r0 = 0; r0 < K8; r0 += 2 * RB) {   // two batches per pass, no copies
                if (r0 + RB < K8) load(vb, vq, r0 + RB);
                accumulate(va, r0);
                if (r0 + RB >= K8) break;
                if (r0 + 2 * RB < K8) load(va, vq, r0 + 2 * RB);
                accumulate(vb, r0 + RB);
            }
            const float av[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int j = j0 + c, i = j - jlo;
                if (i >= 0 && i < nwl) put(i, (j >= 0 && j < S) ? av[c] : NEG);
            }
        }
    } else {
        // Every global value the block needs is requested before any is waited for, so the
        // block pays one memory round trip rather than one per dependent load: the W row
        // over the reachable next states (four loads per thread in flight), then lam_t[k],
        // the stage's normalisation constant V_{t+1}[0][0] and the offset C_{t+1}.
        const float *Wk = a.W + (size_t)k * a.ldw;
        for (int i4 = 0; i4 < nwl; i4 += 4 * NW * 64) {     // nwl > 0: at least one pass
            float w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i4 + u * NW * 64 + tid;
                const int j = jlo + i;
                w[u] = (i < nwl && j >= 0 && j < S) ? Wk[j] : NEG;
            }
            if (i4 == 0) {
                __builtin_amdgcn_sched_barrier(0);      // the scalar loads go out after these
                lam = a.lam[k];
                shift = a.Vn0[0];
                off_next = a.off_next[0];
                if (a.rho1) rsum_m1 = a.rho1[k];
                else if (a.P) rsum_m1 = row_sum_f64(a.P + (size_t)k * a.K, a.K, tid & 63) - 1.0;
                Ad = (float)slope_discharge(lam, a.pay);
                Ac = (float)slope_charge(lam, a.pay);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = i4 + u * NW * 64 + tid;
                if (i < nwl) put(i, w[u]);
            }
        }
    }
    if constexpr (direct) {
        for (int i = tid; i < nchunk * DIRECT_D; i += NW * 64)
            rl[i] = i < span ? move_reward(lam, i - w_down, a.pay) : NEG;
    }
    sweep_sync<NW>();

    const double A_d = slope_discharge(lam, a.pay), A_c = slope_charge(lam, a.pay);
    const double Ct = off_next + (double)shift;   // shift = V_{t+1}[0][0], the normalisation
    // W_t was formed from the normalised V_{t+1}; its true value adds rho_k C_{t+1}, of which
    // C_{t+1} is carried by the offset and (rho_k - 1) C_{t+1} goes into the row (exactly 0
    // when the row sums to 1)
    const double corr = rsum_m1 * off_next - (double)shift;
    const double cst = (double)a.pay.c_start;
    auto emit = [&](int o, double best, int bj) {      // output s0 + o < S
        const int s = s0 + o;
        const float vn = (float)(best + corr);
        const size_t idx = (size_t)k * S + s;
        a.vnorm[(size_t)k * a.ldv + s] = vn;
        // outputs the next launch does not read go out as non-temporal stores
        if (a.vabs) __builtin_nontemporal_store((float)((double)vn + Ct), &a.vabs[idx]);
        if (a.pol) __builtin_nontemporal_store((int16_t)bj, &a.pol[idx]);
        if (a.ckpt_v) __builtin_nontemporal_store(vn, &a.ckpt_v[idx]);
    };
    if constexpr (direct) {
        // Direct maximum over the move range: per output the running maximum of
        // W[j] + r(j - s) in FP32 over chunks of D moves and the first chunk that raised
        // it; that chunk is rescanned for its first move whose candidate (the same
        // operands, so the same bits) equals the maximum: the smallest next state.  The
        // chosen candidate is re-evaluated in FP64 as in the scan path.
        constexpr int R = DIRECT_R, D = DIRECT_D;
        for (int g = tid; g < TS / R; g += NW * 64) {
            const int o0 = g * R;
            float best[R];
            int cid[R];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                best[i] = NEG;
                cid[i] = 0;
            }
            for (int c = 0; c < nchunk; ++c) {
                float w[R + D], r[D];
                const float4 *ws4 = reinterpret_cast<const float4 *>(Wl + o0 + c * D);
                const float4 *rs4 = reinterpret_cast<const float4 *>(rl + c * D);
#pragma unroll
                for (int m = 0; m < (R + D) / 4; ++m) {
                    const float4 v = ws4[m];
                    w[4 * m] = v.x;
                    w[4 * m + 1] = v.y;
                    w[4 * m + 2] = v.z;
                    w[4 * m + 3] = v.w;
                }
#pragma unroll
                for (int m = 0; m < D / 4; ++m) {
                    const float4 v = rs4[m];
                    r[4 * m] = v.x;
                    r[4 * m + 1] = v.y;
                    r[4 * m + 2] = v.z;
                    r[4 * m + 3] = v.w;
                }
#pragma unroll
                for (int i = 0; i < R; ++i) {
                    float m = best[i];
#pragma unroll
                    for (int d = 0; d < D; ++d) m = fmaxf(m, w[i + d] + r[d]);
                    cid[i] = m > best[i] ? c : cid[i];
                    best[i] = m;
                }
            }
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int o = o0 + i;
                if (s0 + o >= S) break;
                const int b = o + cid[i] * D;            // Wl index of the chunk's first move
                int arg = 0;
#pragma unroll
                for (int d = D - 1; d >= 0; --d)
                    arg = Wl[b + d] + rl[cid[i] * D + d] == best[i] ? d : arg;
                const int e = b + arg, dm = e - w_down - o;       // the move j - s
                const double v = dm == 0 ? (double)Wl[e]
                                         : (double)Wl[e] + (dm > 0 ? A_c : A_d) * (double)dm - cst;
                emit(o, v, jlo + e);
            }
        }
        if (k == 0 && tile == 0 && tid == 0) {
            a.off_cur[0] = Ct;
            if (a.ckpt_off) a.ckpt_off[0] = Ct;
        }
        return;
    }

    // Prefix and suffix maxima.  Tasks 0..3 = g_d, h_d, g_c, h_c; with four or more waves
    // each task has NW / 4 waves (two of them split the array at a segment boundary that is
    // a multiple of 8, the segments shifted by phi to make one), with fewer the waves take
    // turns.  Output o reads h(o) and g(o + w - 1).
    {
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        constexpr int G = NW >= 8 ? 2 : 1;
        for (int task = NW >= 4 ? wave / (NW / 4) : wave; task < 4; task += NW >= 4 ? 4 : NW) {
            const int sd = task >> 1;
            const int w = sd ? w_up : w_down;
            if (w == 0) continue;
            const int un = scan_un(TS, w);
            float *const u = sd ? side_c : side_d;
            uint16_t *tg = reinterpret_cast<uint16_t *>(u + un + (task & 1) * scan_tab_words(TS));
            // split point: the multiple of 8 nearest un / 2, made a segment boundary by the
            // shift phi = split mod w (any shift in [0, w) gives segments of w, and the window
            // maxima do not depend on it), so that neither wave runs a pass more than the
            // other for a few entries
            int phi = 0, split = un;
            if (G == 2) {
                const int half = ((un >> 1) + 4) & ~7;
                if (half > 0 && half < un) {
                    split = half;
                    phi = half % w;
                }
            }
            const int gw = NW >= 8 ? wave % 2 : 0;
            if (gw == 1 && split == un) continue;
            const int r0 = gw ? split : 0, r1 = (gw || G == 1) ? un : split;
            if (task & 1)
                window_scan<false>(u, un, w, phi, r0, r1, 0, TS, tg, lane);
            else
                window_scan<true>(u, un, w, phi, r0, r1, scan_glo(w), TS, tg, lane);
        }
    }
    sweep_sync<NW>();

    for (int o = tid; o < TS; o += NW * 64) {
        const int s = s0 + o;
        if (s >= S) break;
        // best candidate of each side: the window's suffix part (smaller next states)
        // wins a tie with its prefix part; j - jlo is the candidate's Wl index
        double best = -INFINITY;
        int bj = s;
        if (w_down) {
            const int un = scan_un(TS, w_down);
            const uint16_t *t = reinterpret_cast<const uint16_t *>(side_d + un);
            const int ph = t[2 * tb + o], pg = t[o + w_down - 1 - scan_glo(w_down)];
            const Cand m = better<true>(table_cand(side_d, un, ph), table_cand(side_d, un, pg));
            if (m.v > NEG) {
                best = (double)Wl[m.e] + A_d * (double)(m.e - w_down - o) - cst;
                bj = jlo + m.e;
            }
        }
        const double idle = (double)Wl[o + w_down];
        if (!(best >= idle)) {
            best = idle;
            bj = s;
        }
        if (w_up) {
            const int un = scan_un(TS, w_up);
            const uint16_t *t = reinterpret_cast<const uint16_t *>(side_c + un);
            const int ph = t[2 * tb + o], pg = t[o + w_up - 1 - scan_glo(w_up)];
            const Cand m = better<true>(table_cand(side_c, un, ph), table_cand(side_c, un, pg));
            if (m.v > NEG) {
                const double v = (double)Wl[w_down + 1 + m.e] + A_c * (double)(m.e + 1 - o) - cst;
                if (v > best) {
                    best = v;
                    bj = s0 + 1 + m.e;
                }
            }
        }
        emit(o, best, bj);
    }
    if (k == 0 && tile == 0 && tid == 0) {
        a.off_cur[0] = Ct;
        if (a.ckpt_off) a.ckpt_off[0] = Ct;
    }
}

// The fields that address a block's first loads (row k of P_t, the first rows of V_{t+1})
// come first as scalar arguments: the library is built to have the first kernel arguments
// preloaded into SGPRs at dispatch, so these loads issue without waiting for a load of the
// argument block (the struct itself is not preloaded).  They override the struct's copies.
template <int NW, bool DIRECT, int RB>
__global__ __launch_bounds__(NW * 64) void sweep_kernel(const float *Vn, const float *lam,
                                                        const float *P, const double *rho1,
                                                        int TS, int ldvn, int K, int S,
                                                        int w_up, int w_down, SweepArgs a)
{
    a.Vn = Vn;
    a.lam = lam;
    a.P = P;
    a.rho1 = rho1;
    a.ldvn = ldvn;
    a.K = K;
    a.S = S;
    a.w_up = w_up;
    a.w_down = w_down;
    extern __shared__ float4 smem4[];
    sweep_block<NW, DIRECT, RB>(a, blockIdx.y, blockIdx.x, TS, reinterpret_cast<float *>(smem4),
                            threadIdx.x);
}

int sweep_tile(const SweepShape &sh) { return sh.TS; }

// Load batch of the fused expectation: 10 rows when that pads K less than 8 does.
static int fused_rows(int K) { return (K + 9) / 10 * 10 - K < (K + 7) / 8 * 8 - K ? 10 : 8; }
// LDS words for row k of P_t padded to its batch (none without the fused expectation)
static size_t fused_prow_words(int K)
{
    if (K <= 0) return 0;
    const int rb = fused_rows(K);
    return (size_t)(((K + rb - 1) / rb * rb + 3) & ~3);
}

size_t sweep_lds_bytes(const SweepShape &sh, int w_up, int w_down, int K)
{
    if (sweep_direct(w_up, w_down)) {
        // the W row with its -inf slack, the reward row, and row k of P_t when fused
        const int span = w_up + w_down + 1;
        const size_t wl = ((size_t)sh.TS + span + DIRECT_D + 3) & ~(size_t)3;
        const size_t rl = (size_t)((span + DIRECT_D - 1) / DIRECT_D) * DIRECT_D;
        return sizeof(float) * (wl + rl + fused_prow_words(K));
    }
    // both sides' u arrays and window tables, the expectation row over the tile's windows
    // (a multiple of 4 entries), and with the fused expectation (K > 0) row k of P_t padded
    // to a multiple of its load batch
    const size_t nwl = ((size_t)sh.TS + w_up + w_down + 3) & ~(size_t)3;
    return sizeof(float) * ((size_t)side_words(sh.TS, w_down) + side_words(sh.TS, w_up) + nwl +
                            fused_prow_words(K));
}

// waves per block with a kernel, and the tile sizes (outputs per block) allowed
#define DP_SWEEP_WAVES(X) X(1) X(2) X(4) X(8)

bool sweep_shape_supported(const SweepShape &sh)
{
    if (sh.TS < 64 || sh.TS > 1024 || sh.TS % 64) return false;
#define X(nw) \
    if (sh.NW == nw) return true;
    DP_SWEEP_WAVES(X)
#undef X
    return false;
}

hipError_t launch_sweep(const SweepArgs &a, const SweepShape &sh, hipStream_t stream)
{
    dim3 grid((a.S + sh.TS - 1) / sh.TS, a.K);
    const size_t lds = sweep_lds_bytes(sh, a.w_up, a.w_down, a.Vn ? a.K : 0);
    const bool direct = sweep_direct(a.w_up, a.w_down);
    const bool rb10 = fused_rows(a.K) == 10;
#define DP_SWEEP_LAUNCH(nw, dr, rb)                                                           \
    hipLaunchKernelGGL((sweep_kernel<nw, dr, rb>), grid, dim3(nw * 64), lds, stream, a.Vn,     \
                       a.lam, a.P, a.rho1, sh.TS, a.ldvn, a.K, a.S, a.w_up, a.w_down, a)
#define X(nw)                                                                                 \
    if (sh.NW == nw) {                                                                        \
        if (direct) {                                                                         \
            if (rb10) DP_SWEEP_LAUNCH(nw, true, 10);                                          \
            else DP_SWEEP_LAUNCH(nw, true, 8);                                                \
        } else {                                                                              \
            if (rb10) DP_SWEEP_LAUNCH(nw, false, 10);                                         \
            else DP_SWEEP_LAUNCH(nw, false, 8);                                               \
        }                                                                                     \
        return hipGetLastError();                                                             \
    }
    DP_SWEEP_WAVES(X)
#undef X
#undef DP_SWEEP_LAUNCH
    return hipErrorInvalidValue;
}

// rho1[t][k] = row_sum_f64(P_t[k]) - 1: one wave per row, the sweep's summation order.
__global__ __launch_bounds__(256) void row_sums_kernel(const float *__restrict__ P, int K,
                                                       int rows, double *__restrict__ rho1)
{
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;                      // per wave: every lane of it leaves together
    const double s = row_sum_f64(P + (size_t)r * K, K, threadIdx.x & 63);
    if ((threadIdx.x & 63) == 0) rho1[r] = s - 1.0;
}

hipError_t launch_row_sums(const float *P, int K, int nstage, double *rho1, hipStream_t stream)
{
    const int rows = K * nstage;
    hipLaunchKernelGGL(row_sums_kernel, dim3((rows + 3) / 4), dim3(256), 0, stream, P, K, rows,
                       rho1);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Stagewise-independent prices on the paper's power grid (Sec. III, Algorithm 1).
//
// One launch per stage.  Block = a tile of TS SoC indices for all R price samples; the
// value row V_t over every next state the tile can reach is staged in LDS once and shared
// by the R samples (in this model the continuation value does not depend on the sample).
// Work unit = (RB consecutive samples, group of G consecutive outputs); the value window
// and move tables of each chunk are read from LDS once for the RB samples.  Per sample and
// output, the interior moves (whole grid
// steps, Algorithm 1's non-interpolated columns) run through the chunked max-plus loop
// with the exact first-argmax rescan; the two endpoint actions +-p_bar (interpolated
// columns) are then compared in next-state order (discharge endpoint first, charge
// endpoint last, strict >), giving the smallest maximising next state.  Q(s, r) goes to
// LDS; V_{t-1}(s) = sum_r pi_r Q(s, r) is formed by NP <= 16 threads per output, thread p
// summing r = p, p + NP, ... in ascending order, and the NP partial sums added in ascending p.
//
// Launch shape (iid_shape): TS = ceil(S / 256) rounded up to a multiple of G, so a stage
// has at most one block per CU; the block has 64 w threads with w chosen so that the
// ceil(R / RB) TS / G units divide as evenly as possible over them.
// ------------------------------------------------------------------------------------
constexpr int IID_D = 8;
constexpr int IID_G = 4;             // outputs per unit
// price samples per unit (they share the LDS reads): 4 when the block still has at least
// four waves of units, else 1 (small grids are latency-bound and need the threads)
constexpr int IID_RB_MAX = 4;

IidShape iid_shape(int R, int S)
{
    IidShape sh;
    const int per = (S + 255) / 256;
    sh.TS = ((per + IID_G - 1) / IID_G) * IID_G;
    const int ngrp = sh.TS / IID_G;
    sh.RB = ((R + IID_RB_MAX - 1) / IID_RB_MAX) * ngrp >= 256 ? IID_RB_MAX : 1;
    const int units = ((R + sh.RB - 1) / sh.RB) * ngrp;
    int best_w = 1;
    double best = 1e30;
    for (int w = 1; w <= 16; ++w) {
        const int n = 64 * w;
        const int iters = (units + n - 1) / n;
        // cost: iterations of the busiest thread, then fewer idle lanes, then more threads
        const double c = iters + 1e-3 * ((double)iters * n - units) / n - 1e-6 * w;
        if (c < best) {
            best = c;
            best_w = w;
        }
    }
    sh.threads = 64 * best_w;
    // partial sums per output: about sqrt(R) balances the two sequential phases
    sh.NP = std::max(1, std::min(sh.threads / sh.TS, 16));
    return sh;
}

// Endpoint tables in FP64 with the formulas of Algorithm 1: sigma = s delta + F(p),
// z = clip(sigma, 0, s_bar) / delta, z- = floor(z + 1e-9), z+ = ceil(z - 1e-9),
// b = (z - z-) / (z+ - z-) (0 when equal), infeasible when sigma < -tol or
// sigma > s_bar + tol, tol = 1e-9 s_bar.
__global__ void iid_tables_kernel(int S, double delta, double eta, double p_bar, IidEnd *endc,
                                  IidEnd *endd)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double s_bar = (double)(S - 1) * delta;
    const double tol = 1e-9 * s_bar;
    for (int side = 0; side < 2; ++side) {
        // charge endpoint p = -p_bar: F = -eta p = eta p_bar; discharge p = +p_bar: F = -p / eta
        const double F = side == 0 ? eta * p_bar : -(p_bar / eta);
        const double sigma = (double)s * delta + F;
        IidEnd e;
        if (sigma < -tol || sigma > s_bar + tol) {
            e.lo = -1;
            e.hi = -1;
            e.b = 0.0f;
        } else {
            const double z = fmin(fmax(sigma, 0.0), s_bar) / delta;
            int lo = (int)floor(z + 1e-9), hi = (int)ceil(z - 1e-9);
            lo = min(lo, hi);
            e.lo = lo;
            e.hi = hi;
            e.b = hi > lo ? (float)((z - lo) / (double)(hi - lo)) : 0.0f;
        }
        (side == 0 ? endc : endd)[s] = e;
    }
}

hipError_t launch_iid_tables(int S, double delta, double eta, double p_bar, IidEnd *endc,
                             IidEnd *endd, hipStream_t stream)
{
    hipLaunchKernelGGL(iid_tables_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, S, delta,
                       eta, p_bar, endc, endd);
    return hipGetLastError();
}

__global__ void iid_init_kernel(float *V, int S, double *off, float *vabs)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S; i += gridDim.x * blockDim.x) {
        V[i] = 0.0f;
        if (vabs) vabs[i] = 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = 0.0;
}

hipError_t launch_iid_init(float *V, int S, double *off, float *vabs, hipStream_t stream)
{
    hipLaunchKernelGGL(iid_init_kernel, dim3((S + 255) / 256), dim3(256), 0, stream, V, S, off,
                       vabs);
    return hipGetLastError();
}

template <int RB>
__global__ __launch_bounds__(1024) void iid_stage_kernel(IidArgs a)
{
    constexpr int D = IID_D, G = IID_G;
    extern __shared__ float4 smem4[];
    float *smem = reinterpret_cast<float *>(smem4);
    const int tid = threadIdx.x, nth = blockDim.x;
    const int S = a.S, R = a.R, TS = a.TS, NP = a.NP;
    const int s0 = blockIdx.x * TS;
    const int s_end = min(s0 + TS, S);
    const int dlo = max(-a.w_down, -(s_end - 1));
    const int dhi = min(a.w_up, S - 1 - s0);
    const int nchunk = (dhi - dlo + 1 + D - 1) / D;
    const int nrl = nchunk * D;
    // LDS: value halo over j in [s0 - w_down - 1, s0 + TS + w_up + 1] (-inf outside [0, S)),
    // reward tables over the tile's interior moves, lam_t and pi_t, Q[R][TS], partial sums
    // [NP][TS].
    const int hb = s0 - a.w_down - 1;                      // first halo index
    const int nh = (TS + a.w_down + a.w_up + 3 + D + 3) & ~3;
    float *Vh = smem;
    float *gl = Vh + nh;
    float *hl = gl + nrl;
    float *pr = hl + nrl;
    float *pl = pr + R;
    float *Q = pl + R;                                     // [R][TS]
    float *part = Q + (size_t)R * TS;                      // [NP][TS]
    const float NEG = -INFINITY;
    // one pass issues every global load (value halo, pi_t, lam_t, and behind them V_t[0]
    // and C_{t+1} for the epilogue) before any is used; nload > TS, so every thread that
    // writes an output makes at least one pass
    const int nload = max(nh, R);
    float shift = 0.0f;
    double off_next = 0.0;
    for (int i = tid; i < nload; i += nth) {
        const int j = hb + i;
        const float v = (i < nh && j >= 0 && j < S) ? a.Vin[j] : NEG;
        const float pv = i < R ? a.prob[i] : 0.0f;
        const float lv = i < R ? a.lam[i] : 0.0f;
        if (i == tid) {
            __builtin_amdgcn_sched_barrier(0);
            shift = a.Vin[0];                              // V_t[0]: the normalisation
            off_next = a.off_next[0];
        }
        if (i < nh) Vh[i] = v;
        if (i < R) {
            pr[i] = pv;
            pl[i] = lv;
        }
    }
    for (int i = tid; i < nrl; i += nth) {
        const int d = dlo + i;
        gl[i] = move_energy(d, a.pay);
        hl[i] = (d <= dhi) ? move_cost(d, a.pay) : NEG;
    }
    __syncthreads();
    const int ngrp = TS / G;
    const int nrb = (R + RB - 1) / RB;
    const int units = nrb * ngrp;
    const int woff = s0 + dlo - hb;                        // halo index of the tile's first next state
    // work unit = (RB consecutive samples, G consecutive outputs): the value window and the
    // move tables of a chunk are read once for the RB samples
    for (int u = tid; u < units; u += nth) {
        const int rb = u / ngrp, grp = u - rb * ngrp;
        const int o0 = grp * G;                            // first output of the group (local)
        const float *Wl = Vh + woff + o0;
        float lamq[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = rb * RB + q;
            lamq[q] = r < R ? pl[r] : 0.0f;
        }
        float best[RB][G];
        int cid[RB][G];
#pragma unroll
        for (int q = 0; q < RB; ++q)
#pragma unroll
            for (int i = 0; i < G; ++i) {
                best[q][i] = NEG;
                cid[q][i] = 0;
            }
        for (int c = 0; c < nchunk; ++c) {
            float w[G + D], gg[D], hh[D];
#pragma unroll
            for (int m = 0; m < G + D - 1; ++m) w[m] = Wl[c * D + m];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                gg[d] = gl[c * D + d];
                hh[d] = hl[c * D + d];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                float rr[D];
#pragma unroll
                for (int d = 0; d < D; ++d) rr[d] = fmaf(lamq[q], gg[d], hh[d]);
#pragma unroll
                for (int i = 0; i < G; ++i) {
                    float m = best[q][i];
#pragma unroll
                    for (int d = 0; d < D; ++d) m = fmaxf(m, w[i + d] + rr[d]);
                    cid[q][i] = (m > best[q][i]) ? c : cid[q][i];
                    best[q][i] = m;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = rb * RB + q;
            if (r >= R) break;
            const float lam = lamq[q];
#pragma unroll
            for (int i = 0; i < G; ++i) {
                const int s = s0 + o0 + i;
                if (s >= S) continue;
                // first interior move attaining the maximum
                int arg = 0;
                for (int d = D - 1; d >= 0; --d) {
                    const float x = Wl[cid[q][i] * D + i + d] +
                                    fmaf(lam, gl[cid[q][i] * D + d], hl[cid[q][i] * D + d]);
                    if (x == best[q][i]) arg = d;
                }
                const int dstar = dlo + cid[q][i] * D + arg;   // interior move (next state s + dstar)
                float qv = best[q][i];
                int act = a.w_up + 1 - dstar;                  // ascending-power index of that move
                // discharge endpoint: smallest next state, wins ties
                const IidEnd ed = a.endd[s];
                if (ed.lo >= 0) {
                    const float vl = Vh[ed.lo - hb], vh = Vh[ed.hi - hb];
                    const float x = fmaf(lam, a.p_bar, (1.0f - ed.b) * vl + ed.b * vh);
                    if (x >= qv) {
                        qv = x;
                        act = a.P - 1;
                    }
                }
                // charge endpoint: largest next state, loses ties
                const IidEnd ec = a.endc[s];
                if (ec.lo >= 0) {
                    const float vl = Vh[ec.lo - hb], vh = Vh[ec.hi - hb];
                    const float x = fmaf(lam, -a.p_bar, (1.0f - ec.b) * vl + ec.b * vh);
                    if (x > qv) {
                        qv = x;
                        act = 0;
                    }
                }
                Q[r * TS + o0 + i] = qv;
                if (a.pol) a.pol[(size_t)r * S + s] = (int16_t)act;
            }
        }
    }
    __syncthreads();
    // expectation: NP partial sums per output (fixed order), then their ordered sum
    for (int x = tid; x < NP * TS; x += nth) {
        const int o = x % TS, p = x / TS;
        float acc = 0.0f;
        for (int r = p; r < R; r += NP) acc = fmaf(pr[r], Q[r * TS + o], acc);
        part[p * TS + o] = acc;
    }
    __syncthreads();
    const double Ct = off_next + (double)shift;
    // the expectation of the offset C_t is (sum_r pi_r) C_t: C_t is carried by the offset,
    // (sum_r pi_r - 1) C_t goes into the values (exactly 0, and skipped, when pi sums to 1)
    const double corr = (row_sum_f64(pr, R, tid & 63) - 1.0) * off_next;
    for (int o = tid; o < TS; o += nth) {
        const int s = s0 + o;
        if (s >= S) continue;
        float acc = part[o];
        for (int p = 1; p < NP; ++p) acc += part[p * TS + o];
        const float vn = corr == 0.0 ? acc - shift : (float)((double)(acc - shift) + corr);
        a.Vout[s] = vn;
        if (a.vabs) a.vabs[s] = (float)((double)vn + Ct);
    }
    if (blockIdx.x == 0 && tid == 0) a.off_cur[0] = Ct;
}

size_t iid_lds_bytes(int R, int S, int w_up, int w_down)
{
    const IidShape sh = iid_shape(R, S);
    const int span = w_up + w_down + 1;
    const int nrl = ((span + IID_D - 1) / IID_D) * IID_D;
    const int nh = (sh.TS + w_down + w_up + 3 + IID_D + 3) & ~3;
    return sizeof(float) * ((size_t)nh + 2 * (size_t)nrl + 2 * (size_t)R + (size_t)R * sh.TS +
                            (size_t)sh.NP * sh.TS);
}

hipError_t launch_iid_stage(const IidArgs &a_in, hipStream_t stream)
{
    const IidShape sh = iid_shape(a_in.R, a_in.S);
    IidArgs a = a_in;
    a.TS = sh.TS;
    a.NP = sh.NP;
    const size_t lds = iid_lds_bytes(a.R, a.S, a.w_up, a.w_down);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid((a.S + sh.TS - 1) / sh.TS);
    if (sh.RB == IID_RB_MAX)
        hipLaunchKernelGGL(iid_stage_kernel<IID_RB_MAX>, grid, dim3(sh.threads), lds, stream, a);
    else
        hipLaunchKernelGGL(iid_stage_kernel<1>, grid, dim3(sh.threads), lds, stream, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Batched solves: every launch covers one batch stage tau of all instances; instance i
// is at its own stage t = T_i - tau + 1 (inactive once t < 1).  The same tile functions
// as the single solve, with arguments taken from the instance descriptor.
// ------------------------------------------------------------------------------------
// One-wave shapes run four independent tiles per block (one per wave, each with its own
// LDS slice of lds_tile floats), so a CU keeps four times as many short tiles in flight.
template <int NW>
constexpr int tiles_per_block() { return NW == 1 ? 4 : 1; }

template <int NW>
__global__ __launch_bounds__(NW * 64 * tiles_per_block<NW>()) void batched_sweep_kernel(
    const BatchDesc *__restrict__ desc, const SweepItem *__restrict__ items, int n, int tau,
    int lds_tile, int TS)
{
    extern __shared__ float4 smem4[];
    constexpr int TPB = tiles_per_block<NW>();
    // the wave's slot is uniform across its lanes; readfirstlane lets the compiler keep the
    // item, its descriptor and every derived address in scalar registers
    const int slot = TPB > 1 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : 0;
    const int item = blockIdx.x * TPB + slot;
    if (item >= n) return;                 // per wave when TPB > 1 (no block barrier then)
    const SweepItem it = items[item];
    const BatchDesc d = desc[it.inst];
    const int t = d.T - tau + 1;
    if (t < 1) return;
    SweepArgs a;
    a.W = d.W;
    a.ldw = d.ld;
    a.lam = d.lam + (size_t)(t - 1) * d.K;
    a.P = d.P ? d.P + (size_t)(t - 1) * d.K * d.K : nullptr;
    a.rho1 = nullptr;
    a.Vn = nullptr;
    a.K = d.K;
    a.S = d.S;
    a.w_up = d.w_up;
    a.w_down = d.w_down;
    a.pay = d.pay;
    const int cur = (d.T - t) & 1;
    a.vnorm = cur ? d.vbuf0 : d.vbuf1;
    a.Vn0 = cur ? d.vbuf1 : d.vbuf0;          // V_{t+1}, read by this stage's expectation
    a.ldv = d.ld;
    a.off_next = d.off + (t + 1);
    a.off_cur = d.off + t;
    a.vabs = (t == 1) ? d.V1 : nullptr;
    a.pol = d.pol ? d.pol + (size_t)(t - 1) * d.K * d.S : nullptr;
    a.ckpt_v = nullptr;
    a.ckpt_off = nullptr;
    float *smem = reinterpret_cast<float *>(smem4) + (size_t)slot * lds_tile;
    const int tid = TPB > 1 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    if (sweep_direct(a.w_up, a.w_down))     // per instance: a class can hold both kinds
        sweep_block<NW, true>(a, it.k, it.tile, TS, smem, tid);
    else
        sweep_block<NW, false>(a, it.k, it.tile, TS, smem, tid);
}

__global__ __launch_bounds__(256) void batched_contract_kernel(const BatchDesc *__restrict__ desc,
                                                               const ContractItem *__restrict__ items,
                                                               int n, int tau)
{
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (wid >= n) return;
    const ContractItem it = items[wid];
    const BatchDesc d = desc[it.inst];
    const int t = d.T - tau + 1;
    if (t < 1) return;
    const float *vin = ((d.T - t) & 1) ? d.vbuf1 : d.vbuf0;
    contract_strip<8, 4>(d.P + (size_t)(t - 1) * d.K * d.K, vin, d.ld, d.W, d.ld, d.K, d.S,
                         it.tm, it.tn);
}

// Column-panel expectation for K <= 128.  An item is `tm` consecutive 64-column panels of
// one instance (field reuse: tm = panel count, tn = first 16-column tile); each wave of the
// block owns one 16-column tile of a panel and walks every row tile.  P_t is staged once
// per item in LDS with a row stride of panel_ld(K) = 4 (mod 32) words, so the 16 rows x 4
// k-offsets a wave reads at once fall in distinct banks; when K % 4 != 0 the columns
// K .. 4 ceil(K/4) - 1 are zero.  The B operands of the next panel are loaded while the
// current panel's MFMAs run (for K <= 64; beyond, the registers would cost occupancy).
// The tile loop is instantiated per k-step count NK = ceil(K/4):
// all NK A operands of a tile are read from LDS ahead of a straight-line chain of NK MFMAs.
// Rows beyond K read row K-1 (their outputs are discarded).  Every tile's chain is exactly
// the tile chain (NK MFMAs in k order on the same operands), so the results are bitwise
// the same.
constexpr int PANEL_KMAX = 128;

__host__ __device__ constexpr int panel_ld(int K) { return ((K + 31) / 32) * 32 + 4; }

template <int NK>
__device__ __forceinline__ void panel_load_b(const float *__restrict__ B, int ldb, int K,
                                             int col, bool cok, float (&bv)[NK])
{
    const int kq = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int i = 0; i < NK; ++i) {
        const int kx = 4 * i + kq;
        bv[i] = (kx < K && cok) ? B[(size_t)kx * ldb + col] : 0.f;
    }
}

template <int NK, bool PREFETCH>
__device__ __forceinline__ void panel_run(const float *__restrict__ Pl, int ldp, int K, int S,
                                          const float *__restrict__ B, int ldb,
                                          float *__restrict__ W, int ldw, int tn0, int npan)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, kq = lane >> 4;
    const int ntm = (K + 15) >> 4;
    int col = (tn0 + wave) * 16 + (lane & 15);
    float bv[NK];
    panel_load_b<NK>(B, ldb, K, col, col < S, bv);
    for (int pn = 0; pn < npan; ++pn) {
        const bool cok = col < S;
        const int ncol = col + 64;
        float bn[NK];
        if (PREFETCH && pn + 1 < npan) panel_load_b<NK>(B, ldb, K, ncol, ncol < S, bn);
        for (int tm = 0; tm < ntm; ++tm) {
            const int arow = tm * 16 + (lane & 15);
            const float *ap = Pl + (arow < K ? arow : K - 1) * ldp + kq;
            // A operands in groups of 8 k-steps: group g + 1 is read while group g's MFMAs
            // run (the scheduling barriers keep that order)
            constexpr int NG = (NK + 7) / 8;
            float av[NK];
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (g == 0) {
#pragma unroll
                    for (int i = 0; i < 8 && i < NK; ++i) av[i] = ap[4 * i];
                }
                if (g + 1 < NG) {
#pragma unroll
                    for (int i = 8 * (g + 1); i < 8 * (g + 2) && i < NK; ++i) av[i] = ap[4 * i];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 8 * g; i < 8 * (g + 1) && i < NK; ++i)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i], acc, 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (cok) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int r = tm * 16 + 4 * kq + v;
                    if (r < K) W[(size_t)r * ldw + col] = acc[v];
                }
            }
        }
        if (pn + 1 < npan) {
            if (PREFETCH) {
#pragma unroll
                for (int i = 0; i < NK; ++i) bv[i] = bn[i];
            } else {
                panel_load_b<NK>(B, ldb, K, ncol, ncol < S, bv);
            }
        }
        col = ncol;
    }
}

// One instantiation per k-step class [NKLO, NKHI] (1-8, 9-16, 17-32), so each launch
// carries only the registers its own k range needs.
template <int NKLO, int NKHI>
__global__ __launch_bounds__(256) void batched_panel_kernel(const BatchDesc *__restrict__ desc,
                                                            const ContractItem *__restrict__ items,
                                                            int tau)
{
    extern __shared__ float4 smem4[];
    float *Pl = reinterpret_cast<float *>(smem4);
    const ContractItem it = items[blockIdx.x];
    const BatchDesc d = desc[it.inst];
    const int t = d.T - tau + 1;
    if (t < 1) return;
    const int K = d.K, S = d.S, ldp = panel_ld(K);
    const float *P = d.P + (size_t)(t - 1) * K * K;
    const int tid = threadIdx.x;
    if ((K & 3) == 0 && (reinterpret_cast<uintptr_t>(P) & 15) == 0) {
        // rows of K / 4 float4s, eight loads in flight per thread
        const int k4 = K >> 2, n4 = K * k4;
        const float4 *src = reinterpret_cast<const float4 *>(P);
        for (int e0 = 0; e0 < n4; e0 += 8 * 256) {
            // indices past the end are clamped to the last element: the same value is
            // loaded and stored to the same place again, so no lane needs a branch
            int e[8], o[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                e[u] = min(e0 + u * 256 + tid, n4 - 1);
                const int r = e[u] / k4;
                o[u] = r * ldp + 4 * (e[u] - r * k4);
            }
            const float4 v0 = src[e[0]], v1 = src[e[1]], v2 = src[e[2]], v3 = src[e[3]];
            const float4 v4 = src[e[4]], v5 = src[e[5]], v6 = src[e[6]], v7 = src[e[7]];
            float4 *dst = reinterpret_cast<float4 *>(Pl);
            dst[o[0] >> 2] = v0; dst[o[1] >> 2] = v1; dst[o[2] >> 2] = v2; dst[o[3] >> 2] = v3;
            dst[o[4] >> 2] = v4; dst[o[5] >> 2] = v5; dst[o[6] >> 2] = v6; dst[o[7] >> 2] = v7;
        }
    } else {
        const int kp = ((K + 3) >> 2) << 2;     // zero columns K .. kp - 1
        for (int e0 = 0; e0 < K * kp; e0 += 4 * 256) {
            float v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * 256 + tid;
                const int r = e / kp, c = e - r * kp;
                v[u] = (e < K * kp && c < K) ? P[(size_t)r * K + c] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = e0 + u * 256 + tid;
                const int r = e / kp, c = e - r * kp;
                if (e < K * kp) Pl[r * ldp + c] = v[u];
            }
        }
    }
    __syncthreads();
    const float *B = ((d.T - t) & 1) ? d.vbuf1 : d.vbuf0;
    switch ((K + 3) >> 2) {
#define DP_PANEL_CASE(n)                                                                    \
    case n:                                                                                 \
        if constexpr (n >= NKLO && n <= NKHI)                                               \
            panel_run<n, (NKHI <= 16)>(Pl, ldp, K, S, B, d.ld, d.W, d.ld, it.tn, it.tm);    \
        break;
        DP_PANEL_CASE(1) DP_PANEL_CASE(2) DP_PANEL_CASE(3) DP_PANEL_CASE(4)
        DP_PANEL_CASE(5) DP_PANEL_CASE(6) DP_PANEL_CASE(7) DP_PANEL_CASE(8)
        DP_PANEL_CASE(9) DP_PANEL_CASE(10) DP_PANEL_CASE(11) DP_PANEL_CASE(12)
        DP_PANEL_CASE(13) DP_PANEL_CASE(14) DP_PANEL_CASE(15) DP_PANEL_CASE(16)
        DP_PANEL_CASE(17) DP_PANEL_CASE(18) DP_PANEL_CASE(19) DP_PANEL_CASE(20)
        DP_PANEL_CASE(21) DP_PANEL_CASE(22) DP_PANEL_CASE(23) DP_PANEL_CASE(24)
        DP_PANEL_CASE(25) DP_PANEL_CASE(26) DP_PANEL_CASE(27) DP_PANEL_CASE(28)
        DP_PANEL_CASE(29) DP_PANEL_CASE(30) DP_PANEL_CASE(31) DP_PANEL_CASE(32)
#undef DP_PANEL_CASE
        default: break;
    }
}

int panel_class(int K) { return K <= 32 ? 0 : (K <= 64 ? 1 : 2); }

hipError_t launch_batched_panel(const BatchDesc *desc, const ContractItem *items, int n, int tau,
                                int kmax, hipStream_t stream)
{
    const size_t lds = sizeof(float) * (size_t)kmax * panel_ld(kmax);
    switch (panel_class(kmax)) {
        case 0:
            hipLaunchKernelGGL((batched_panel_kernel<1, 8>), dim3(n), dim3(256), lds, stream, desc, items, tau);
            break;
        case 1:
            hipLaunchKernelGGL((batched_panel_kernel<9, 16>), dim3(n), dim3(256), lds, stream, desc, items, tau);
            break;
        default:
            hipLaunchKernelGGL((batched_panel_kernel<17, 32>), dim3(n), dim3(256), lds, stream, desc, items, tau);
            break;
    }
    return hipGetLastError();
}

__global__ void batched_init_kernel(const BatchDesc *__restrict__ desc)
{
    const BatchDesc d = desc[blockIdx.y];
    const size_t n = (size_t)d.K * d.ld;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        d.vbuf0[i] = 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) d.off[d.T + 1] = 0.0;
}

hipError_t launch_batched_init(const BatchDesc *desc, int n, hipStream_t stream)
{
    hipLaunchKernelGGL(batched_init_kernel, dim3(64, n), dim3(256), 0, stream, desc);
    return hipGetLastError();
}

hipError_t launch_batched_contract(const BatchDesc *desc, const ContractItem *items, int n,
                                   int tau, hipStream_t stream)
{
    hipLaunchKernelGGL(batched_contract_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, desc,
                       items, n, tau);
    return hipGetLastError();
}

int batched_tiles_per_block(const SweepShape &sh) { return sh.NW == 1 ? tiles_per_block<1>() : 1; }

hipError_t launch_batched_sweep(const BatchDesc *desc, const SweepItem *items, int n, int tau,
                                const SweepShape &sh, size_t lds, hipStream_t stream)
{
    // lds: one tile's bytes; a block of tiles_per_block tiles gets one 16-byte aligned
    // slice each
    const int lds_tile = (int)(((lds + 15) & ~(size_t)15) / sizeof(float));
#define X(nw)                                                                                \
    if (sh.NW == nw) {                                                                       \
        constexpr int tpb = tiles_per_block<nw>();                                           \
        hipLaunchKernelGGL((batched_sweep_kernel<nw>), dim3((n + tpb - 1) / tpb),            \
                           dim3(nw * 64 * tpb), (size_t)lds_tile * sizeof(float) * tpb,      \
                           stream, desc, items, n, tau, lds_tile, sh.TS);                    \
        return hipGetLastError();                                                            \
    }
    DP_SWEEP_WAVES(X)
#undef X
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------
// Terminal state: normalised values = src (v_term, a checkpoint, or 0) with offset
// *src_off (or 0); optional absolute copy (float)(value + offset).
// ------------------------------------------------------------------------------------
__global__ void init_terminal_kernel(const float *src, const double *src_off, int K, int S,
                                     float *vnorm, int ldv, double *off, float *vabs)
{
    const double o = src_off ? src_off[0] : 0.0;
    const size_t n = (size_t)K * S;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i / S), s = (int)(i % S);
        const float v = src ? src[i] : 0.0f;
        vnorm[(size_t)k * ldv + s] = v;
        if (vabs) vabs[i] = (float)((double)v + o);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) off[0] = o;
}

hipError_t launch_init_terminal(const float *src, const double *src_off, int K, int S,
                                float *vnorm, int ldv, double *off, float *vabs,
                                hipStream_t stream)
{
    const size_t n = (size_t)K * S;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(init_terminal_kernel, dim3(blocks), dim3(256), 0, stream, src, src_off,
                       K, S, vnorm, ldv, off, vabs);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Adjoint: push the occupation measure through the policy (deterministic).
//
// nu_t[k][j] = sum_{s: pi_t[k][s] = j} mu_t[k][s] is accumulated in LDS as 64-bit fixed
// point: each mass is scaled by a power of two 2^e (exact), rounded once to an integer,
// and added with ds_add_u64.  Integer addition is associative, so the sums do not depend
// on the order the lanes reach LDS.  2^e is chosen from a bound B on sum |mu| (the adjoint
// is mass-preserving under row-stochastic P, so B = 2 sum |seed| bounds every stage):
// 2^e B <= 2^61 keeps every partial sum inside int64, and the rounding of each mass is at
// most 2^-62 B.  grad_lam[k] = sum_s mu[s] g(pi(s) - s) uses per-lane sums, a fixed
// butterfly within each wave and the waves' sums in wave order.  One block per price
// state; the block's policy and mass loads (up to PF per thread) and the scale are issued
// before the accumulator is cleared, so the block waits for one memory round trip.
// The accumulator covers PUSH_JC next states at a time (128 KB of LDS): rows longer than
// that take one pass per chunk of next states, each over every s.  A policy entry outside
// [0, S) adds nothing (memory safety; dp_adjoint with DP_VALIDATE rejects such policies).
// ------------------------------------------------------------------------------------
constexpr int PF = 8;
constexpr int PUSH_JC = 16384;

__global__ __launch_bounds__(1024) void pushforward_kernel(const float *__restrict__ mu,
                                                           int ldm,
                                                           const int16_t *__restrict__ pol,
                                                           int K, int S, Payoff pay,
                                                           const double *__restrict__ scale,
                                                           float *__restrict__ nu, int ldn,
                                                           float *__restrict__ grad_lam)
{
    extern __shared__ float4 smem4[];
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem4);   // [min(S, JC)]
    __shared__ float red[16];
    const int k = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int16_t *pk = pol + (size_t)k * S;
    const float *mk = mu + (size_t)k * ldm;
    int jv[PF];
    float mv[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        const int s = tid + u * nt;
        jv[u] = s < S ? pk[s] : 0;
        mv[u] = s < S ? mk[s] : 0.0f;
    }
    const double sc = scale[0];
    const double inv = 1.0 / sc;
    float gl = 0.0f;
    for (int j0 = 0; j0 < S; j0 += PUSH_JC) {
        const int jn = min(PUSH_JC, S - j0);
        for (int i = tid; i < jn; i += nt) acc[i] = 0ull;
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int s = tid + u * nt;
            if (s < S) {
                if (j0 == 0) gl = fmaf(mv[u], move_energy(jv[u] - s, pay), gl);
                const unsigned jr = (unsigned)(jv[u] - j0);
                if (jr < (unsigned)jn)
                    atomicAdd(&acc[jr], (unsigned long long)llrint((double)mv[u] * sc));
            }
        }
        for (int s = tid + PF * nt; s < S; s += nt) {      // beyond the preloaded elements
            const int j = pk[s];
            const float m = mk[s];
            if (j0 == 0) gl = fmaf(m, move_energy(j - s, pay), gl);
            const unsigned jr = (unsigned)(j - j0);
            if (jr < (unsigned)jn) atomicAdd(&acc[jr], (unsigned long long)llrint((double)m * sc));
        }
        __syncthreads();
        for (int i = tid; i < jn; i += nt)
            nu[(size_t)k * ldn + j0 + i] = (float)((double)(long long)acc[i] * inv);
        __syncthreads();                                    // acc is cleared next pass
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gl += __shfl_xor(gl, o);
    if ((tid & 63) == 0) red[tid >> 6] = gl;
    __syncthreads();
    if (tid == 0) {
        float sum = red[0];
        for (int w = 1; w < (nt >> 6); ++w) sum += red[w];
        grad_lam[k] = sum;
    }
}

hipError_t launch_pushforward(const float *mu, int ldm, const int16_t *pol, int K, int S,
                              Payoff pay, const double *scale, float *nu, int ldn,
                              float *grad_lam, hipStream_t stream)
{
    const size_t lds = sizeof(unsigned long long) * (size_t)min(S, PUSH_JC);
    const int nt = S >= 4096 ? 1024 : (S >= 1024 ? 512 : 256);
    hipLaunchKernelGGL(pushforward_kernel, dim3(K), dim3(nt), lds, stream, mu, ldm, pol, K, S,
                       pay, scale, nu, ldn, grad_lam);
    return hipGetLastError();
}

// Policy check for dp_adjoint with DP_VALIDATE: every entry a feasible next state,
// max(0, s - w_down) <= j <= min(S - 1, s + w_up); *flag is set to 1 otherwise.
__global__ void validate_policy_kernel(const int16_t *__restrict__ pol, size_t n, int S,
                                       int w_up, int w_down, int *flag)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(i % S), j = pol[i];
        if (j < max(0, s - w_down) || j > min(S - 1, s + w_up)) atomicOr(flag, 1);
    }
}

hipError_t launch_validate_policy(const int16_t *pol, size_t n, int S, int w_up, int w_down,
                                  int *flag, hipStream_t stream)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(validate_policy_kernel, dim3(blocks), dim3(256), 0, stream, pol, n, S,
                       w_up, w_down, flag);
    return hipGetLastError();
}

// Power-of-two fixed-point scale for the push-forward from the seed:
// B = 2 sum |seed| (fixed-order tree in one block), scale = 2^floor(log2(2^61 / B)).
__global__ __launch_bounds__(1024) void adjoint_scale_kernel(const float *__restrict__ seed,
                                                             size_t n, double *scale)
{
    __shared__ double red[1024];
    double a = 0.0;
    for (size_t i = threadIdx.x; i < n; i += 1024) a += fabs((double)seed[i]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double B = fmax(2.0 * red[0], 1e-300);
        int e;
        frexp(B, &e);                       // B < 2^e
        scale[0] = ldexp(1.0, 61 - e);      // 2^(61 - e) B < 2^61
    }
}

hipError_t launch_adjoint_scale(const float *seed, size_t n, double *scale, hipStream_t stream)
{
    hipLaunchKernelGGL(adjoint_scale_kernel, dim3(1), dim3(1024), 0, stream, seed, n, scale);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// grad_P_t = nu_t V_{t+1}^T for a group of consecutive stages (one launch per group; the
// transport mu_{t+1} = P_t^T nu_t is the expectation kernel with A = P^T, per stage).
// A block = one 16 x 16 tile of one stage of the group, 16 waves: wave w reduces the
// w-th sixteenth of j (one chunk of prefetched MFMA steps), and the 16 partial tiles are
// added in wave order, so each gradient entry has one fixed summation order.
// ------------------------------------------------------------------------------------
constexpr int GRADP_WAVES = 16;

__global__ __launch_bounds__(64 * GRADP_WAVES) void gradP_kernel(
    const float *__restrict__ nu0, size_t nu_stride, int ldn, const float *__restrict__ V0,
    size_t v_stride, int K, int S, int G, float *__restrict__ gP0)
{
    constexpr int CH = 16;
    __shared__ float part[GRADP_WAVES][256];
    // Blocks are dealt to the 8 XCDs in turn by index: block 8 i + x runs on XCD x.  Stage g
    // of the group takes XCD g mod 8, so all its tiles read its rows of nu and V through one
    // L2 (a stage spread over every XCD had each L2 fetch them: 7x the algorithmic bytes).
    const int ntm = (K + 15) >> 4, nt2 = ntm * ntm;
    const int xcd = blockIdx.x & 7, bi = blockIdx.x >> 3;
    const int g = xcd + 8 * (bi / nt2), tile = bi % nt2;
    if (g >= G) return;                        // the whole block: past the group's stages
    const float *nu = nu0 + g * nu_stride;
    const float *V = V0 + g * v_stride;
    float *gP = gP0 + (size_t)g * K * K;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tm = tile % ntm, tn = tile / ntm;
    const int kq = lane >> 4;
    const int arow = tm * 16 + (lane & 15);   // k
    const int bcol = tn * 16 + (lane & 15);   // k'
    const bool rok = arow < K, cok = bcol < K;
    const int steps = (S + 3) / 4;
    const int per = (steps + GRADP_WAVES - 1) / GRADP_WAVES;
    const int jb = wave * per * 4, je = min(S, (wave + 1) * per * 4);
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int j0 = jb; j0 < je; j0 += 4 * CH) {
        float av[CH], bv[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int j = j0 + 4 * i + kq;
            const bool jok = j < je;
            av[i] = (jok && rok) ? nu[(size_t)arow * ldn + j] : 0.f;
            bv[i] = (jok && cok) ? V[(size_t)bcol * S + j] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < CH; ++i)
            if (j0 + 4 * i < je) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[i], acc, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) part[wave][(4 * kq + v) * 16 + (lane & 15)] = acc[v];
    __syncthreads();
    if (tid < 256) {
        const int r = tid >> 4, c = tid & 15;
        const int kr = tm * 16 + r, kc = tn * 16 + c;
        float sum = part[0][tid];
#pragma unroll
        for (int w = 1; w < GRADP_WAVES; ++w) sum += part[w][tid];
        if (kr < K && kc < K) gP[(size_t)kr * K + kc] = sum;
    }
}

hipError_t launch_gradP(const float *nu, size_t nu_stride, int ldn, const float *V,
                        size_t v_stride, int K, int S, int G, float *gP, hipStream_t stream)
{
    const int nt = (K + 15) / 16;
    // one block per (stage, tile), stages grouped by XCD (8 blocks per tile slot)
    hipLaunchKernelGGL(gradP_kernel, dim3(8 * nt * nt * ((G + 7) / 8)), dim3(64 * GRADP_WAVES),
                       0, stream, nu, nu_stride, ldn, V, v_stride, K, S, G, gP);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Small utilities.
// ------------------------------------------------------------------------------------
__global__ void copy_rows_kernel(const float *src, int lds, float *dst, int ldd, int K, int S)
{
    const size_t n = (size_t)K * S;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(i / S), s = (int)(i % S);
        dst[(size_t)k * ldd + s] = src[(size_t)k * lds + s];
    }
}

hipError_t launch_copy_rows(const float *src, int lds, float *dst, int ldd, int K, int S,
                            hipStream_t stream)
{
    const size_t n = (size_t)K * S;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(copy_rows_kernel, dim3(blocks), dim3(256), 0, stream, src, lds, dst, ldd,
                       K, S);
    return hipGetLastError();
}

__global__ void fill_kernel(float *dst, size_t n, float v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = v;
}

hipError_t launch_fill(float *dst, size_t n, float v, hipStream_t stream)
{
    int blocks = (int)((n + 255) / 256);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, stream, dst, n, v);
    return hipGetLastError();
}

// Row check of the transition tensor: every entry >= 0 and |row sum - 1| <= 1e-6.
__global__ void validate_P_kernel(const float *P, int T, int K, int *flag)
{
    const size_t rows = (size_t)T * K;
    for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < rows;
         r += (size_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        bool neg = false;
        for (int c = 0; c < K; ++c) {
            const float v = P[r * K + c];
            neg |= !(v >= 0.0f);
            sum += (double)v;
        }
        if (neg || fabs(sum - 1.0) > 1e-6) atomicOr(flag, 1);
    }
}

hipError_t launch_validate_P(const float *P, int T, int K, int *flag, hipStream_t stream)
{
    const size_t rows = (size_t)T * K;
    int blocks = (int)((rows + 255) / 256);
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(validate_P_kernel, dim3(blocks), dim3(256), 0, stream, P, T, K, flag);
    return hipGetLastError();
}

}  // namespace dpk
