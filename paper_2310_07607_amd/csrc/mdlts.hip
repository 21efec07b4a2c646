// mdlts.hip -- the C ABI (include/mdlts.h) and the non-substep kernels:
// CFL + level assignment, stable grouping by level, table remapping, state
// permutation, FP64 error indicator, refinement transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "abi_guard.hpp"
#include "amr.hpp"
#include "host.hpp"
#include "kernels.hpp"
#include "variants.hpp"
#include "mdlts.h"

using namespace mdlts;

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return MDLTS_EDEVICE; \
    } while (0)
#define MD_TRY(x)                           \
    do {                                    \
        mdlts_status _s = (x);              \
        if (_s != MDLTS_OK) return _s;      \
    } while (0)

namespace {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// level assignment (Sec. 2.3: Gershgorin CFL per element, b^CFL) and the
// stable grouping of elements by level, finest first
// ---------------------------------------------------------------------------
struct LevelArgs {
    const void *key;
    const uint32_t *face;  // canonical [2d][E]
    int E;
    int dim;
    int n_levels;
    double dt_bar;
    double h0[3];
    double Dk[3];
    double G[4][4];
    const double *otab;  // full tensors: root bound per face-kind combination, else null
    int force_level;  // >= 0: every leaf on this level (no CFL test)
    const double *eta_t;  // RV-T indicator per leaf, or null: no cell criterion
    double tau_cell;      // threshold of the cell criterion
    int b_cell;           // level the criterion asks for
    uint8_t *level;
    double *cfl;
    int *hist;      // [blocks][8]
    int *bad;       // set if some leaf needs more levels than configured
};

template <int DIM, typename A = LevelArgs>
// (A: the arguments by value from a kernel parameter, by reference from an op table)
__device__ __forceinline__ void levels_body(const int blk, A a)
{
#pragma clang fp contract(off)
    __shared__ int sh[kMaxLevels];
    if (threadIdx.x < kMaxLevels) sh[threadIdx.x] = 0;
    __syncthreads();
    const int e = blk * kBlock + threadIdx.x;
    if (e < a.E) {
        int depth;
        uint32_t c[3];
        unpack_key<DIM>(static_cast<const typename KeyOf<DIM>::type *>(a.key)[e], depth, c);
        double s = 0.0;
        if (a.otab) {
            // full tensor: the own block couples the directions; its bound
            // is the root's for these face kinds, times 4^depth (exact)
            uint32_t idx = 0;
            for (int f = 0; f < 2 * DIM; f++) idx |= (a.face[(long long)f * a.E + e] >> 30) << (2 * f);
            s = a.otab[idx] * ldexp(1.0, 2 * depth);
        } else {
            for (int k = 0; k < DIM; k++) {
                const double h = ldexp(a.h0[k], -depth);
                const uint32_t lo = a.face[(long long)(2 * k) * a.E + e] >> 30;
                const uint32_t hi = a.face[(long long)(2 * k + 1) * a.E + e] >> 30;
                s += a.Dk[k] / (h * h) * a.G[lo][hi];
            }
        }
        const double cfl = 1.0 / s;
        int b = 0;
        if (a.force_level >= 0) b = a.force_level;
        else
            while (b < 64 && ldexp(a.dt_bar, -b) > cfl) b++;
        // the cell criterion (RV-T indicator above its threshold)
        if (a.eta_t && a.force_level < 0 && a.eta_t[e] > a.tau_cell && a.b_cell > b) b = a.b_cell;
        if (b > a.n_levels - 1) {
            atomicOr(a.bad, 1);
            b = a.n_levels - 1;
        }
        a.level[e] = (uint8_t)b;
        a.cfl[e] = cfl;
        atomicAdd(&sh[b], 1);
    }
    __syncthreads();
    if (threadIdx.x < kMaxLevels) a.hist[blk * kMaxLevels + threadIdx.x] = sh[threadIdx.x];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_levels(const LevelArgs a)
{
    levels_body<DIM>(blockIdx.x, a);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct LevelsOp {
    LevelArgs a;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        levels_body<DIM, const LevelArgs &>(blk, a);
    }
};

// smallest of n positive doubles: wavefront minimum, one atomic per wave
// (for positive doubles the bit patterns order like the values)
__global__ __launch_bounds__(kBlock) void k_min_positive(int n, const double *x, unsigned long long *min_bits)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    double m = i < n ? x[i] : 1.0e308;
    for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMin(min_bits, (unsigned long long)__double_as_longlong(m));
}

// exclusive offsets of every (block, level) in the finest-first order
__device__ __forceinline__ void level_scan_body(const int blk, int *hist, int nb, int n_levels, int *cnt_ge, int *cnt_ge2)
{
    __shared__ int wtot[kBlock / 64][kMaxLevels];
    __shared__ int base[kMaxLevels];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int chunk = (nb + kBlock - 1) / kBlock;
    const int b0 = t * chunk, b1 = min(nb, b0 + chunk);
    // this thread's rows, summed per level, then scanned over the block's
    // threads: wavefront inclusive scans by shuffles, then the waves' totals
    int excl[kMaxLevels];
#pragma unroll
    for (int l = 0; l < kMaxLevels; l++) {
        int v = 0;
        for (int b = b0; b < b1; b++) v += hist[b * kMaxLevels + l];
        int x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wtot[wave][l] = x;
        excl[l] = x - v;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < kMaxLevels; l++)
        for (int w = 0; w < wave; w++) excl[l] += wtot[w][l];
    if (t == 0) {
        int run = 0;
        for (int l = kMaxLevels - 1; l >= 0; l--) {
            int tot = 0;  // leaves of level l
            for (int w = 0; w < kBlock / 64; w++) tot += wtot[w][l];
            base[l] = run;  // leaves of finer levels come first
            run += tot;
            cnt_ge[l] = l < n_levels ? run : 0;  // every entry written
            if (cnt_ge2) cnt_ge2[l] = cnt_ge[l];  // a second copy (readback block)
        }
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < kMaxLevels; l++) {
        int run = base[l] + excl[l];
        for (int b = b0; b < b1; b++) {
            const int v = hist[b * kMaxLevels + l];
            hist[b * kMaxLevels + l] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_level_scan(int *hist, int nb, int n_levels, int *cnt_ge, int *cnt_ge2)
{
    level_scan_body(blockIdx.x, hist, nb, n_levels, cnt_ge, cnt_ge2);
}

// its arguments, for a launch over many simulations (k_multi)
struct LevelScanOp {
    int *hist;
    int nb;
    int n_levels;
    int *cnt_ge;
    int *cnt_ge2;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        level_scan_body(blk, hist, nb, n_levels, cnt_ge, cnt_ge2);
    }
};

// position of every element: block offset + rank among equal levels inside
// the block (wavefront ballots keep the canonical order: stable)
__device__ __forceinline__ void level_scatter_body(const int blk, const uint8_t *level, int E, const int *off, int *perm,
                                                          int *inv)
{
    __shared__ int wcount[kBlock / 64][kMaxLevels];
    const int e = blk * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int l = e < E ? level[e] : -1;
    int rank = 0;
    for (int q = 0; q < kMaxLevels; q++) {
        const unsigned long long m = __ballot(l == q);
        if (lane == 0) wcount[wave][q] = __popcll(m);
        if (l == q) rank = __popcll(m & ((1ull << lane) - 1ull));
    }
    __syncthreads();
    if (e < E) {
        int pos = off[blk * kMaxLevels + l] + rank;
        for (int w = 0; w < wave; w++) pos += wcount[w][l];
        perm[pos] = e;
        inv[e] = pos;
    }
}

__global__ __launch_bounds__(kBlock) void k_level_scatter(const uint8_t *level, int E, const int *off, int *perm,
                                                          int *inv)
{
    level_scatter_body(blockIdx.x, level, E, off, perm, inv);
}

// its arguments, for a launch over many simulations (k_multi)
struct LevelScatterOp {
    const uint8_t *level;
    int E;
    const int *off;
    int *perm;
    int *inv;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        level_scatter_body(blk, level, E, off, perm, inv);
    }
};

template <typename KT, int NS>
__device__ __forceinline__ void remap_body(const int blk, int E, int nfaces, const int *perm, const int *inv,
                                                  const uint8_t *level, const KT *key_c, const uint32_t *face_c,
                                                  const uint32_t *fine_c, KT *key_s, uint32_t *nbr_s,
                                                  uint32_t *fine_s, int cap)
{
    const int j = blk * kBlock + threadIdx.x;
    if (j >= E) return;
    const int e = perm[j];
    key_s[j] = key_c[e];
    for (int f = 0; f < nfaces; f++) {
        const uint32_t ent = face_c[(long long)f * E + e];
        const uint32_t kind = ent >> 30;
        uint32_t out = ent & 0xc0000000u;
        if (kind == kSame || kind == kCoarser) {
            const uint32_t n = ent & kIdMask30;
            out |= ((uint32_t)level[n] << 27) | (uint32_t)inv[n];
        } else if (kind == kFiner) {
            for (int q = 0; q < NS; q++) {
                const uint32_t n = fine_c[((long long)f * E + e) * NS + q];
                fine_s[((long long)f * cap + j) * NS + q] = ((uint32_t)level[n] << 27) | (uint32_t)inv[n];
            }
        }
        nbr_s[(long long)f * cap + j] = out;
    }
}

template <typename KT, int NS>
__global__ __launch_bounds__(kBlock) void k_remap(int E, int nfaces, const int *perm, const int *inv,
                                                  const uint8_t *level, const KT *key_c, const uint32_t *face_c,
                                                  const uint32_t *fine_c, KT *key_s, uint32_t *nbr_s,
                                                  uint32_t *fine_s, int cap)
{
    remap_body<KT, NS>(blockIdx.x, E, nfaces, perm, inv, level, key_c, face_c, fine_c, key_s, nbr_s, fine_s, cap);
}

// its arguments, for a launch over many simulations (k_multi)
template <typename KT, int NS>
struct RemapOp {
    int E;
    int nfaces;
    const int *perm;
    const int *inv;
    const uint8_t *level;
    const KT *key_c;
    const uint32_t *face_c;
    const uint32_t *fine_c;
    KT *key_s;
    uint32_t *nbr_s;
    uint32_t *fine_s;
    int cap;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        remap_body<KT, NS>(blk, E, nfaces, perm, inv, level, key_c, face_c, fine_c, key_s, nbr_s, fine_s, cap);
    }
};

// canonical [np][E] -> grouped slot 0 [np][cap]
template <typename T>
__device__ __forceinline__ void permute_body(const int blk, int E, int np, int cap, const int *perm, const T *uc, const T *vc,
                                                    T *us, T *vs)
{
    const int j = blk * kBlock + threadIdx.x;
    if (j >= E) return;
    const int e = perm[j];
    // grouped layout (grp_elem, grp_node): blocks of 64 elements with
    // [node][element] inside a block, [node][cap] for Q1 quadrilaterals
    const long long gj = np == 4 ? j : (long long)(j >> 6) * np * 64 + (j & 63);
    const long long gn = np == 4 ? cap : 64;
    for (int n = 0; n < np; n++) {
        us[gj + (long long)n * gn] = uc[(long long)n * E + e];
        vs[gj + (long long)n * gn] = vc[(long long)n * E + e];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(int E, int np, int cap, const int *perm, const T *uc, const T *vc,
                                                    T *us, T *vs)
{
    permute_body<T>(blockIdx.x, E, np, cap, perm, uc, vc, us, vs);
}

// its arguments, for a launch over many simulations (k_multi)
template <typename T>
struct PermuteOp {
    int E;
    int np;
    int cap;
    const int *perm;
    const T *uc;
    const T *vc;
    T *us;
    T *vs;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        permute_body<T>(blk, E, np, cap, perm, uc, vc, us, vs);
    }
};

// grouped current slot -> canonical [np][E] (at a barrier)
template <typename T>
__device__ __forceinline__ void gather_body(const int blk, int E, int np, int cap, long long slot_stride, const int *perm,
                                                   const int *cnt_ge, int parity, const T *us, const T *vs, T *uc,
                                                   T *vc, int *zero32)
{
    // (zero32, if given: 32 ints cleared by the first block, for the
    // kernels that follow on the stream)
    if (zero32 && blk == 0 && threadIdx.x < 32) zero32[threadIdx.x] = 0;
    const int j = blk * kBlock + threadIdx.x;
    if (j >= E) return;
    // level-0 elements sit at the end of the grouped order
    const bool lvl0 = j >= cnt_ge[1];
    const int cur = lvl0 ? parity : 0;
    const int e = perm[j];
    // grouped layout (grp_elem, grp_node)
    const long long gj = np == 4 ? j : (long long)(j >> 6) * np * 64 + (j & 63);
    const long long gn = np == 4 ? cap : 64;
    for (int n = 0; n < np; n++) {
        uc[(long long)n * E + e] = us[(long long)cur * slot_stride + gj + (long long)n * gn];
        if (vc) vc[(long long)n * E + e] = vs[gj + (long long)n * gn];
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_gather(int E, int np, int cap, long long slot_stride, const int *perm,
                                                   const int *cnt_ge, int parity, const T *us, const T *vs, T *uc,
                                                   T *vc, int *zero32)
{
    gather_body<T>(blockIdx.x, E, np, cap, slot_stride, perm, cnt_ge, parity, us, vs, uc, vc, zero32);
}

// its arguments, for a launch over many simulations (k_multi)
template <typename T>
struct GatherOp {
    int E;
    int np;
    int cap;
    long long slot_stride;
    const int *perm;
    const int *cnt_ge;
    int parity;
    const T *us;
    const T *vs;
    T *uc;
    T *vc;
    int *zero32;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        gather_body<T>(blk, E, np, cap, slot_stride, perm, cnt_ge, parity, us, vs, uc, vc, zero32);
    }
};

// clears n 32-bit words (a kernel rather than a memset, so that the
// clearing is an ordinary kernel node if the caller captures the stream)
__global__ __launch_bounds__(64) void k_clear_u32(uint32_t *p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// host FP64 [E][np] <-> device T [np][E]
template <typename T>
__global__ __launch_bounds__(kBlock) void k_from_host(int E, int np, const double *h, T *d)
{
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)E * np) return;
    const long long e = q / np, n = q % np;
    d[n * E + e] = (T)h[q];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_to_host(int E, int np, const T *d, double *h)
{
    const long long q = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (q >= (long long)E * np) return;
    const long long e = q / np, n = q % np;
    h[q] = (double)d[n * E + e];
}

// ---------------------------------------------------------------------------
// Kelly-type indicator (Sec. 2.2), FP64 accumulation, canonical layout
// ---------------------------------------------------------------------------
struct IndArgs {
    const void *u;  // canonical [np][E], bulk precision
    const void *key;
    const uint32_t *face;
    const uint32_t *fine;
    int E;
    int p;
    double h0[3];
    double Dk[3];
    double Dx[3];  // off-diagonal Dxy, Dxz, Dyz
    int full;      // some off-diagonal entry is nonzero
    DevRef<double> ref;
    double *eta;
    unsigned long long *eta_max_bits;
    int *nonfinite;
};

template <int DIM, int P, typename T>
__device__ __forceinline__ void canon_trace(const IndArgs &a, uint32_t id, int k, int side, double *tu, double *tq)
{
    using S = Shape<DIM, P>;
    const T *u = static_cast<const T *>(a.u);
#pragma unroll
    for (int g = 0; g < S::NF; g++) {
        double su = 0.0, sq = 0.0;
#pragma unroll
        for (int b = 0; b < S::M; b++) {
            const double val = (double)u[(long long)fnode<DIM, S::M>(k, g, b) * a.E + id];
            su += a.ref.B[side][b] * val;
            sq += a.ref.G[side][b] * val;
        }
        tu[g] = su;
        tq[g] = sq;
    }
}

// Tangential part of the jump of n.D grad u at the face points: with a full
// tensor, n.D grad u = ns sum_t D_kt d/dx_t u + the normal part.  The traces
// are given at the points of the (sub-)face, whose reference coordinates
// scale by `scale` / h_t (2 on a face, 4 on a half-size sub-face).
template <int DIM, int M, bool FULL>
__device__ __forceinline__ void tangential_jump(const IndArgs &a, const RefConst &R, int k, double ns, double scale,
                                                const double *h, const double *tu, const double *nu, double *tj)
{
    constexpr int NF = DIM == 2 ? M : M * M;
    for (int g = 0; g < NF; g++) tj[g] = 0.0;
    if constexpr (!FULL) return;
    double df[NF], d[NF];
    for (int g = 0; g < NF; g++) df[g] = tu[g] - nu[g];
    for (int tau = 0; tau < DIM - 1; tau++) {
        const int t = tang_dir(k, tau);
        face_line<double, DIM, M>(R.D1, tau, df, d);
        const double c = ns * a.Dx[off_slot(k, t)] * scale / h[t];
        for (int g = 0; g < NF; g++) tj[g] += c * d[g];
    }
}

template <int DIM, int P, typename T, bool FULL, typename A = IndArgs>
// (A: the arguments by value from a kernel parameter, by reference from an op table)
__device__ __forceinline__ void indicator_body(const int blk, A a)
{
    using S = Shape<DIM, P>;
    constexpr int M = S::M, NF = S::NF, NS = S::NS;
    constexpr RefConst R = ref_const(P);
    const int e = blk * kBlock + threadIdx.x;
    double eta = 0.0;
    if (e < a.E) {
        int depth;
        uint32_t c[3] = {0, 0, 0};
        unpack_key<DIM>(static_cast<const typename KeyOf<DIM>::type *>(a.key)[e], depth, c);
        double h[3] = {1, 1, 1};
        for (int k = 0; k < DIM; k++) h[k] = ldexp(a.h0[k], -depth);
        // face entries first; Q1 quadrilaterals also take every same-size or
        // coarser neighbour's trace up front (16 doubles), so the faces do not
        // wait for memory one after another (same arithmetic, same results)
        uint32_t ents[2 * DIM];
#pragma unroll
        for (int f = 0; f < 2 * DIM; f++) ents[f] = a.face[(long long)f * a.E + e];
        constexpr bool kPre = 2 * DIM * NF * 2 <= 16;
        double pu[kPre ? 2 * DIM : 1][NF], pq[kPre ? 2 * DIM : 1][NF];
        if constexpr (kPre) {
#pragma unroll
            for (int f = 0; f < 2 * DIM; f++) {
                const uint32_t kind = ents[f] >> 30;
                if (kind == kSame || kind == kCoarser)
                    canon_trace<DIM, P, T>(a, ents[f] & kIdMask30, f >> 1, 1 - (f & 1), pu[f], pq[f]);
            }
        }
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; k++) {
            int pos0 = 0, pos1 = 0, t = 0;
            double area = 1.0;
            for (int q = 0; q < DIM; q++) {
                if (q == k) continue;
                if (t == 0) pos0 = c[q] & 1; else pos1 = c[q] & 1;
                area *= h[q];
                t++;
            }
            // reference weights of the tangential GL rule on [0,1]^(d-1)
            double om[NF];
#pragma unroll
            for (int g = 0; g < NF; g++)
                om[g] = DIM == 2 ? 0.5 * a.ref.w[g] : 0.25 * a.ref.w[g % M] * a.ref.w[g / M];
#pragma unroll
            for (int s = 0; s < 2; s++) {
                const uint32_t ent = ents[2 * k + s];
                const uint32_t kind = ent >> 30;
                if (kind == kBoundary) continue;
                const double ns = s ? 1.0 : -1.0;
                const double qs = ns * a.Dk[k] * 2.0 / h[k];
                double tu[NF], tq[NF];
                canon_trace<DIM, P, T>(a, (uint32_t)e, k, s, tu, tq);
                if (kind != kFiner) {
                    double nu[NF], nq[NF];
                    if constexpr (kPre) {
                        for (int g = 0; g < NF; g++) {
                            nu[g] = pu[2 * k + s][g];
                            nq[g] = pq[2 * k + s][g];
                        }
                    } else {
                        canon_trace<DIM, P, T>(a, ent & kIdMask30, k, 1 - s, nu, nq);
                    }
                    const double hn = kind == kSame ? h[k] : 2.0 * h[k];
                    if (kind == kCoarser) {
                        double iq[NF], iu[NF];
                        tang_apply<double, DIM, M>(a.ref.Isub, pos0, pos1, nq, iq);
                        tang_apply<double, DIM, M>(a.ref.Isub, pos0, pos1, nu, iu);
                        for (int g = 0; g < NF; g++) { nq[g] = iq[g]; nu[g] = iu[g]; }
                    }
                    const double qn = ns * a.Dk[k] * 2.0 / hn;
                    double tj[NF];
                    tangential_jump<DIM, M, FULL>(a, R, k, ns, 2.0, h, tu, nu, tj);
                    double integral = 0.0;
                    for (int g = 0; g < NF; g++) {
                        const double jmp = qs * tq[g] - qn * nq[g] + tj[g];
                        integral += om[g] * area * jmp * jmp;
                    }
                    const double hF = DIM == 2 ? area : sqrt(area);
                    acc += hF / (2.0 * a.p) * area * area * integral;
                } else {
                    const double sarea = DIM == 2 ? 0.5 * area : 0.25 * area;
                    const double hF = DIM == 2 ? sarea : sqrt(sarea);
                    const double qn = ns * a.Dk[k] * 2.0 / (0.5 * h[k]);
                    for (int sub = 0; sub < NS; sub++) {
                        double oq[NF], ou[NF], nu[NF], nq[NF], tj[NF];
                        tang_apply<double, DIM, M>(a.ref.Isub, sub & 1, sub >> 1, tq, oq);
                        tang_apply<double, DIM, M>(a.ref.Isub, sub & 1, sub >> 1, tu, ou);
                        canon_trace<DIM, P, T>(a, a.fine[((long long)(2 * k + s) * a.E + e) * NS + sub], k, 1 - s, nu, nq);
                        tangential_jump<DIM, M, FULL>(a, R, k, ns, 4.0, h, ou, nu, tj);
                        double integral = 0.0;
                        for (int g = 0; g < NF; g++) {
                            const double jmp = qs * oq[g] - qn * nq[g] + tj[g];
                            integral += om[g] * sarea * jmp * jmp;
                        }
                        acc += hF / (2.0 * a.p) * sarea * sarea * integral;
                    }
                }
            }
        }
        eta = sqrt(acc);
        a.eta[e] = eta;
        if (!isfinite(eta)) atomicOr(a.nonfinite, 1);
    }
    // block maximum through wavefront shuffles, one atomic per wave
    double m = isfinite(eta) ? eta : 0.0;
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(a.eta_max_bits, (unsigned long long)__double_as_longlong(m));
}

template <int DIM, int P, typename T, bool FULL>
__global__ __launch_bounds__(kBlock) void k_indicator(const IndArgs a)
{
    indicator_body<DIM, P, T, FULL>(blockIdx.x, a);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM, int P, typename T, bool FULL>
struct IndicatorOp {
    IndArgs a;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        indicator_body<DIM, P, T, FULL, const IndArgs &>(blk, a);
    }
};

// ---------------------------------------------------------------------------
// RV-T temporal indicator (Sec. 2.3): per element, over a barrier [t_a, t_b],
// the L2 norms over [t_a, t_b] x e of the changes of the ionic current I and
// of the gate rate g since t_a, divided by t_b - t_a.  The time integrals use
// the midpoint rule at the state linear in time between the barrier's end
// values (the S-LTS representation of a coarse element between its
// updates); I includes the stimulus.  FP64 from the bulk-precision states.
// ---------------------------------------------------------------------------
struct RvtArgs {
    const void *u_a, *v_a;  // canonical [np][E], bulk precision: state at t_a
    const void *u_b, *v_b;  // the same at t_b
    const void *key;
    int E;
    double h0[3];
    double apk, apa, eps0, mu1, mu2;
    double t_a, t_b;
    int n_stim;
    double stim[kMaxStim][9];
    double *eta;
    unsigned long long *eta_max_bits;
};

__device__ __forceinline__ double rvt_current(const RvtArgs &a, double u, double v)
{
    return -a.apk * u * (u - a.apa) * (u - 1.0) - u * v;
}

__device__ __forceinline__ double rvt_gate_rate(const RvtArgs &a, double u, double v)
{
    double den = u + a.mu2;
    den = den < 1e-6 ? 1e-6 : den;
    const double eps = a.eps0 + a.mu1 * v / den;
    return eps * (a.apk * u * (1.0 + a.apa - u) - v);
}

__device__ __forceinline__ double rvt_stimulus(const RvtArgs &a, const double *X, int dim, double t)
{
    double s = 0.0;
    for (int b = 0; b < a.n_stim; b++) {
        bool in = t >= a.stim[b][6] && t < a.stim[b][7];
        for (int k = 0; k < dim; k++) in = in && X[k] >= a.stim[b][k] && X[k] <= a.stim[b][3 + k];
        if (in) s += a.stim[b][8];
    }
    return s;
}

template <int DIM, int P, typename T>
__global__ __launch_bounds__(kBlock) void k_rvt(const RvtArgs a)
{
    using S = Shape<DIM, P>;
    constexpr int M = S::M, NP = S::NP;
    constexpr RefConst R = ref_const(P);
    const int e = blockIdx.x * kBlock + threadIdx.x;
    double eta = 0.0;
    if (e < a.E) {
        int depth;
        uint32_t c[3] = {0, 0, 0};
        unpack_key<DIM>(static_cast<const typename KeyOf<DIM>::type *>(a.key)[e], depth, c);
        double h[3] = {1, 1, 1}, lo[3] = {0, 0, 0};
        for (int k = 0; k < DIM; k++) {
            h[k] = ldexp(a.h0[k], -depth);
            lo[k] = (double)c[k] * h[k];
        }
        const double t_m = 0.5 * (a.t_a + a.t_b);
        const T *ua = static_cast<const T *>(a.u_a), *va = static_cast<const T *>(a.v_a);
        const T *ub = static_cast<const T *>(a.u_b), *vb = static_cast<const T *>(a.v_b);
        double sum = 0.0;
        for (int n = 0; n < NP; n++) {
            const long long q = (long long)n * a.E + e;
            const double u0 = (double)ua[q], v0 = (double)va[q];
            const double um = 0.5 * (u0 + (double)ub[q]), vm = 0.5 * (v0 + (double)vb[q]);
            double X[3] = {0, 0, 0}, w = 1.0;
            int nn = n;
            for (int k = 0; k < DIM; k++) {
                X[k] = lo[k] + 0.5 * (R.xi[nn % M] + 1.0) * h[k];
                w *= R.w[nn % M] * 0.5 * h[k];  // diagonal mass: GL weight x |J|
                nn /= M;
            }
            const double dI = (rvt_current(a, um, vm) + rvt_stimulus(a, X, DIM, t_m)) -
                              (rvt_current(a, u0, v0) + rvt_stimulus(a, X, DIM, a.t_a));
            const double dg = rvt_gate_rate(a, um, vm) - rvt_gate_rate(a, u0, v0);
            sum += w * (dI * dI + dg * dg);
        }
        eta = sqrt(sum / (a.t_b - a.t_a));
        a.eta[e] = eta;
    }
    double m = isfinite(eta) ? eta : 0.0;
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(a.eta_max_bits, (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------------------
// refinement transfer: copy, prolongation by evaluation, L2 restriction
// ---------------------------------------------------------------------------
struct XferArgs {
    const void *u_old, *v_old;
    void *u_new, *v_new;
    int E_old, E_new;
    const uint8_t *kind;
    const int32_t *src;
    const uint8_t *child;
    DevRef<double> ref;
};

template <int DIM, int P, typename T, typename A = XferArgs>
// (A: the arguments by value from a kernel parameter, by reference from an op table)
__device__ __forceinline__ void transfer_body(const int blk, A a)
{
    using S = Shape<DIM, P>;
    constexpr int M = S::M, NP = S::NP;
    const int e = blk * kBlock + threadIdx.x;
    if (e >= a.E_new) return;
    const int kind = a.kind[e], src = a.src[e], ci = a.child[e];
    for (int f = 0; f < 2; f++) {
        const T *in = static_cast<const T *>(f ? a.v_old : a.u_old);
        T *out = static_cast<T *>(f ? a.v_new : a.u_new);
        if (kind == 0) {
            for (int n = 0; n < NP; n++) out[(long long)n * a.E_new + e] = in[(long long)n * a.E_old + src];
            continue;
        }
        for (int n = 0; n < NP; n++) {
            int nk[3] = {n % M, (n / M) % M, n / (M * M)};
            double s = 0.0;
            const int nkids = kind == 1 ? 1 : (1 << DIM);
            for (int cc = 0; cc < nkids; cc++) {
                const int bits = kind == 1 ? ci : cc;
                for (int q = 0; q < NP; q++) {
                    int qk[3] = {q % M, (q / M) % M, q / (M * M)};
                    double wgt = 1.0;
                    for (int k = 0; k < DIM; k++) {
                        const int bit = (bits >> k) & 1;
                        wgt *= kind == 1 ? a.ref.Isub[bit][nk[k]][qk[k]] : a.ref.Lsub[bit][nk[k]][qk[k]];
                    }
                    s += wgt * (double)in[(long long)q * a.E_old + src + (kind == 1 ? 0 : cc)];
                }
            }
            out[(long long)n * a.E_new + e] = (T)s;
        }
    }
}

template <int DIM, int P, typename T>
__global__ __launch_bounds__(kBlock) void k_transfer(const XferArgs a)
{
    transfer_body<DIM, P, T>(blockIdx.x, a);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM, int P, typename T>
struct TransferOp {
    XferArgs a;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        transfer_body<DIM, P, T, const XferArgs &>(blk, a);
    }
};

inline int nblocks(long long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

// ---------------------------------------------------------------------------
// The scratch memory of the allocation-free indicator (mdlts_indicator_noalloc):
// one fixed device array per GPU, held from the library's load on that GPU to
// the end of the process.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address is taken once per device with
// hipGetSymbolAddress (kept in scratch_dev) and only that address is passed
// to kernels.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices];  // device address of `scratch` per device, set once

// the device address of `scratch` on the current device (`device`)
mdlts_status scratch_address(int device, void **out)
{
    if (device < 0 || device >= kMaxDevices) return MDLTS_EINVAL;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return MDLTS_EDEVICE;
        }
        scratch_dev[device] = p;
    }
    *out = scratch_dev[device];
    return MDLTS_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// context and simulation objects
// ---------------------------------------------------------------------------
struct BatchPlan;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct mdlts_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    void *scratch = nullptr;  // device address of this device's `scratch`
    mdlts_allocator alloc{};
    bool has_alloc = false;
    int n_sims = 0;  // live simulations; the context outlives them
    BatchPlan *batch = nullptr;
    int use_graphs = 1;
    // launch shapes chosen by the autotuner, per mix of kernel variants
    // (bit 12*full + 6*(dim-2) + 2*(order-1) + precision)
    struct Tuned {
        std::map<int, int> blocks;  // variant bit -> threads per block
        int block;                  // that of the variant with the most device time
        double dof;  // DoF-updates per barrier of the plan it was tuned on
        bool single_graph;
    };
    std::map<int, Tuned> tuned;  // mask -> launch shape
    // pinned host staging of plan and constant uploads (copies from it are
    // asynchronous); stage_done follows the last copies out of it
    void *stage = nullptr;
    size_t stage_bytes = 0;
    hipEvent_t stage_done = nullptr;
    // completed synchronisations of the stream: work enqueued before the
    // last one has finished
    uint64_t sync_epoch = 0;
    // launches over many simulations: their op tables (pinned staging and the
    // device copy), and the flags blocks of every simulation collected for one
    // readback
    void *multi_host = nullptr;
    size_t multi_host_bytes = 0;
    DevBuf multi_dev;
    void *flags_host = nullptr;
    size_t flags_host_bytes = 0;
    DevBuf flags_dev;
};

// Host-visible staging of a simulation's small readbacks (pinned memory, so
// the copies into it are asynchronous and one synchronisation can cover the
// readbacks of many simulations).
struct PinnedReadback {
    unsigned long long tallies[3];  // adaptation: refined, coarsened, (spare)
    int total;                      // adaptation: number of new leaves
    int face_bad;                   // face tables: inconsistent mesh
    int level_bad;                  // levels: a leaf needs more levels than configured
    int eta_nonfinite;              // indicator: non-finite values
    unsigned long long eta_max_bits;
    int cnt_ge[kMaxLevels];
};

struct mdlts_sim {
    mdlts_ctx *ctx = nullptr;
    PinnedReadback *pin = nullptr;
    mdlts_mesh_desc desc{};
    int np = 0;
    size_t tsize = 8;  // bytes of the bulk precision
    Forest forest;                 // host mirror of the leaves (lazily refreshed)
    bool host_forest_valid = true;
    size_t E = 0;                  // number of leaves
    RefTables ref{};
    double h0[3] = {1, 1, 1};
    double Dk[3] = {1e-3, 1e-3, 1e-3};
    double Dx[3] = {0.0, 0.0, 0.0};  // off-diagonal Dxy, Dxz, Dyz
    bool dfull = false;              // some off-diagonal entry is nonzero
    double gamma = 2.0;
    double G[4][4] = {};
    // full tensors: own-block Gershgorin bound of a root per face-kind
    // combination (own_block_table), and its device copy
    std::vector<double> otab;
    bool otab_dirty = false;
    DevBuf otab_d;
    mdlts_ap_params ap{8.0, 0.15, 0.002, 0.2, 0.3};
    std::vector<mdlts_stim_box> stim;
    // canonical device data
    DevBuf key_c, face_c, fine_c, u_c, v_c, level_c, cfl_c, eta_c, tmp_u, tmp_v;
    // grouped device data
    DevBuf u_s, v_s, key_s, nbr_s, fine_s, perm, inv, hist, cnt_ge_d, flags, xk, xs, xc, stage;
    // substep constants in device memory and their host copy
    DevBuf step_dev;
    std::vector<unsigned char> step_host = std::vector<unsigned char>(sizeof(StepArgs<double>));
    bool step_dirty = true;
    uint64_t version = 1;  // bumped by every change a batch plan depends on
    // device mesh management
    DevBuf root_start, mkey, refine, cflag, cnt, off, bsums, key_n;
    int cap = 0;
    bool state_grouped = false;  // else canonical
    bool levels_valid = false;
    // the current levels are the CFL levels of dt_bar (no forced level, no
    // cell criterion); the value is set when an assignment completes
    bool levels_plain = false, levels_plain_pending = false;
    std::vector<int32_t> cnt_ge;  // [n_levels]
    int lmax = 0;
    double dt_bar = 0.0;
    double t_start = 0.0;
    long long n_bar = 0;  // barriers since t_start (time bookkeeping)
    // RV-T temporal indicator: state snapshot at t_a and the indicator, each
    // valid for the tree revision it was taken on
    uint64_t tree_rev = 1;  // bumped whenever the leaves change
    DevBuf snap_u, snap_v, eta_t_c;
    double snap_t = 0.0;
    uint64_t snap_rev = 0, eta_t_rev = 0;
    BatchPlan *solo = nullptr;  // graph plan of mdlts_step
    long long n_since_assign = 0;
    uint64_t dof_updates = 0;
    bool eta_valid = false;  // eta_c holds the indicator of the current forest
    // optional event timing of every substep launch
    bool prof = false;
    std::vector<hipEvent_t> ev;  // pairs: start, stop
    size_t ev_used = 0;          // pairs recorded and not yet read
    double prof_ms = 0.0;
    uint64_t prof_launches = 0, prof_dof = 0;
};

namespace {

mdlts_status dev_free(mdlts_ctx *c, DevBuf &b)
{
    if (b.p) {
        if (c->has_alloc) c->alloc.free(b.p, c->stream, c->alloc.user);
        else if (hipFree(b.p) != hipSuccess) return MDLTS_EDEVICE;
    }
    b.p = nullptr;
    b.bytes = 0;
    return MDLTS_OK;
}

mdlts_status dev_alloc(mdlts_ctx *c, DevBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes) return MDLTS_OK;
    MD_TRY(dev_free(c, b));
    if (bytes == 0) bytes = 256;
    // a buffer that grows gets 1/8 more than asked, so that leaf counts that
    // move by a few per cent between adaptations do not go back to the
    // allocator every time (the memory bound includes this headroom)
    bytes += bytes / 8;
    void *p = nullptr;
    if (c->has_alloc) {
        p = c->alloc.alloc(bytes, c->stream, c->alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (!p) return MDLTS_ENOMEM;
    b.p = p;
    b.bytes = bytes;
    return MDLTS_OK;
}

// A simulation's device flags block holds the small readbacks at the
// offsets they have in PinnedReadback, so that each phase writes its own
// fields and one copy brings back what several phases wrote.
constexpr size_t kFlagBytes = 128;
static_assert(kFlagBytes == 32 * sizeof(int), "the gather clears the flags block as 32 ints");
constexpr size_t kFlagHead = offsetof(PinnedReadback, cnt_ge);
static_assert(sizeof(PinnedReadback) <= kFlagBytes, "flags block holds the readback fields");

template <typename F>
F *flag_at(mdlts_sim *s, size_t off)
{
    return reinterpret_cast<F *>(static_cast<char *>(s->flags.p) + off);
}
#define MD_FLAG(s, F, field) flag_at<F>(s, offsetof(PinnedReadback, field))

// zero the whole flags block (every phase's fields)
mdlts_status flags_clear(mdlts_sim *s)
{
    MD_TRY(dev_alloc(s->ctx, s->flags, kFlagBytes));
    HIP_TRY(hipMemsetAsync(s->flags.p, 0, kFlagBytes, s->ctx->stream));
    return MDLTS_OK;
}

// the fields of the flags block into the pinned readback (the level counts
// too when `levels`: a level assignment wrote them); they arrive after the
// next synchronisation
mdlts_status flags_readback(mdlts_sim *s, bool levels = false)
{
    HIP_TRY(hipMemcpyAsync(s->pin, s->flags.p, levels ? sizeof(PinnedReadback) : kFlagHead, hipMemcpyDeviceToHost,
                           s->ctx->stream));
    return MDLTS_OK;
}

// The context's pinned staging area, at least `bytes` long, once the copies
// out of it that were queued before have completed.
mdlts_status stage_acquire(mdlts_ctx *c, size_t bytes, char **out)
{
    if (c->stage_done) {
        HIP_TRY(hipEventSynchronize(c->stage_done));
    } else {
        HIP_TRY(hipEventCreateWithFlags(&c->stage_done, hipEventDisableTiming));
    }
    if (c->stage_bytes < bytes) {
        if (c->stage) (void)hipHostFree(c->stage);
        c->stage = nullptr;
        c->stage_bytes = 0;
        const size_t nb = std::max(bytes + bytes / 4, (size_t)1 << 20);  // headroom for growth
        if (hipHostMalloc(&c->stage, nb, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->stage = nullptr;
            return MDLTS_ENOMEM;
        }
        c->stage_bytes = nb;
    }
    *out = static_cast<char *>(c->stage);
    return MDLTS_OK;
}

// marks the staging area busy until the copies queued so far are done
mdlts_status stage_release(mdlts_ctx *c)
{
    HIP_TRY(hipEventRecord(c->stage_done, c->stream));
    return MDLTS_OK;
}

template <typename T>
T *P(DevBuf &b)
{
    return static_cast<T *>(b.p);
}

template <typename T>
void fill_ref(const RefTables &R, DevRef<T> &D)
{
    std::memset(&D, 0, sizeof(D));
    for (int a = 0; a < kMaxM; a++) {
        D.w[a] = (T)R.w[a];
        D.winv[a] = a < R.m ? (T)(1.0 / R.w[a]) : (T)0;
        D.xi[a] = R.xi[a];
        for (int b = 0; b < kMaxM; b++) D.A[a][b] = (T)R.A[a][b];
    }
    for (int s = 0; s < 2; s++)
        for (int b = 0; b < kMaxM; b++) {
            D.B[s][b] = (T)R.B[s][b];
            D.G[s][b] = (T)R.G[s][b];
            for (int q = 0; q < kMaxM; q++) {
                D.Isub[s][b][q] = (T)R.Isub[s][b][q];
                D.Lsub[s][b][q] = (T)R.Lsub[s][b][q];
            }
        }
}

bool valid_desc(const mdlts_mesh_desc *d)
{
    if (!d) return false;
    if (d->dim != 2 && d->dim != 3) return false;
    if (d->order < 1 || d->order > 3) return false;
    if (d->max_depth < 0 || d->max_depth > 8) return false;
    if (d->n_levels < 1 || d->n_levels > kMaxLevels) return false;
    if (d->precision != MDLTS_FP64 && d->precision != MDLTS_FP32) return false;
    const int bits = d->dim == 2 ? 14 : 20;
    long long roots = 1;
    for (int k = 0; k < d->dim; k++) {
        if (d->n[k] < 1 || !(d->len[k] > 0.0) || !std::isfinite(d->len[k])) return false;
        if (((long long)d->n[k] << d->max_depth) > (1ll << bits)) return false;
        roots *= d->n[k];
    }
    return roots < (1ll << 26);
}

void forest_from_desc(const mdlts_mesh_desc *d, Forest &F)
{
    F.dim = d->dim;
    F.max_depth = d->max_depth;
    for (int k = 0; k < 3; k++) F.n[k] = k < d->dim ? d->n[k] : 1;
}

mdlts_status sync(mdlts_ctx *c)
{
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MDLTS_EDEVICE;
    c->sync_epoch++;
    if (hipGetLastError() != hipSuccess) return MDLTS_EDEVICE;
    return MDLTS_OK;
}

template <typename T>
mdlts_status copy_h2d(mdlts_ctx *c, DevBuf &b, const T *src, size_t n)
{
    MD_TRY(dev_alloc(c, b, n * sizeof(T)));
    if (n) HIP_TRY(hipMemcpyAsync(b.p, src, n * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return MDLTS_OK;
}

MeshGeo geo_of(const mdlts_sim *s)
{
    MeshGeo g;
    for (int k = 0; k < 3; k++) g.n[k] = s->desc.n[k];
    g.max_depth = s->desc.max_depth;
    return g;
}

int n_sub(const mdlts_sim *s) { return s->desc.dim == 2 ? 2 : 4; }

// face tables of the canonical leaves in key_c, built on the device; the
// consistency flag arrives in pin->face_bad after the next synchronisation
mdlts_status device_faces(mdlts_sim *s, bool own_flags = true)
{
    mdlts_ctx *c = s->ctx;
    const int E = (int)s->E;
    const int dim = s->desc.dim;
    const int n_roots = s->desc.n[0] * s->desc.n[1] * (dim == 3 ? s->desc.n[2] : 1);
    MD_TRY(dev_alloc(c, s->root_start, (size_t)(n_roots + 1) * sizeof(int)));
    MD_TRY(dev_alloc(c, s->mkey, (size_t)E * sizeof(uint32_t)));
    MD_TRY(dev_alloc(c, s->face_c, (size_t)2 * dim * E * sizeof(uint32_t)));
    MD_TRY(dev_alloc(c, s->fine_c, (size_t)2 * dim * E * n_sub(s) * sizeof(uint32_t)));
    if (own_flags) MD_TRY(flags_clear(s));
    int *bad = MD_FLAG(s, int, face_bad);
    const MeshGeo g = geo_of(s);
    if (dim == 2) {
        k_mesh_index<2><<<nblocks(E), kBlock, 0, c->stream>>>(E, n_roots, g, P<uint32_t>(s->key_c),
                                                               P<int>(s->root_start), P<uint32_t>(s->mkey));
        k_mesh_faces<2><<<nblocks(2ll * 2 * E), kBlock, 0, c->stream>>>(E, g, P<uint32_t>(s->key_c), P<int>(s->root_start),
                                                               P<uint32_t>(s->mkey), P<uint32_t>(s->face_c),
                                                               P<uint32_t>(s->fine_c), bad);
    } else {
        k_mesh_index<3><<<nblocks(E), kBlock, 0, c->stream>>>(E, n_roots, g, P<uint64_t>(s->key_c),
                                                               P<int>(s->root_start), P<uint32_t>(s->mkey));
        k_mesh_faces<3><<<nblocks(2ll * 3 * E), kBlock, 0, c->stream>>>(E, g, P<uint64_t>(s->key_c), P<int>(s->root_start),
                                                               P<uint32_t>(s->mkey), P<uint32_t>(s->face_c),
                                                               P<uint32_t>(s->fine_c), bad);
    }
    HIP_TRY(hipGetLastError());
    if (own_flags) HIP_TRY(hipMemcpyAsync(&s->pin->face_bad, bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return MDLTS_OK;
}

// face tables and their consistency check, synchronously
mdlts_status device_faces_sync(mdlts_sim *s)
{
    MD_TRY(device_faces(s));
    MD_TRY(sync(s->ctx));
    return s->pin->face_bad ? MDLTS_EINVAL : MDLTS_OK;
}

// upload the leaf keys of the host forest and build the face tables
mdlts_status upload_forest(mdlts_sim *s)
{
    mdlts_ctx *c = s->ctx;
    const Forest &F = s->forest;
    const size_t E = F.size();
    s->E = E;
    s->host_forest_valid = true;
    if (s->desc.dim == 2) {
        std::vector<uint32_t> key(E);
        for (size_t e = 0; e < E; e++) key[e] = pack_key<2>(F.leaves[e].depth, F.leaves[e].c);
        MD_TRY(copy_h2d(c, s->key_c, key.data(), E));
        MD_TRY(sync(c));
    } else {
        std::vector<uint64_t> key(E);
        for (size_t e = 0; e < E; e++) key[e] = pack_key<3>(F.leaves[e].depth, F.leaves[e].c);
        MD_TRY(copy_h2d(c, s->key_c, key.data(), E));
        MD_TRY(sync(c));
    }
    return device_faces_sync(s);
}

// refresh the host mirror of the leaves from the device keys
mdlts_status refresh_host_forest(mdlts_sim *s)
{
    if (s->host_forest_valid) return MDLTS_OK;
    mdlts_ctx *c = s->ctx;
    const size_t E = s->E;
    Forest &F = s->forest;
    forest_from_desc(&s->desc, F);
    F.leaves.resize(E);
    if (s->desc.dim == 2) {
        std::vector<uint32_t> key(E);
        HIP_TRY(hipMemcpyAsync(key.data(), s->key_c.p, E * 4, hipMemcpyDeviceToHost, c->stream));
        MD_TRY(sync(c));
        for (size_t e = 0; e < E; e++) {
            F.leaves[e].depth = (uint8_t)(key[e] & 15);
            F.leaves[e].c[0] = (key[e] >> 4) & 0x3fff;
            F.leaves[e].c[1] = (key[e] >> 18) & 0x3fff;
            F.leaves[e].c[2] = 0;
        }
    } else {
        std::vector<uint64_t> key(E);
        HIP_TRY(hipMemcpyAsync(key.data(), s->key_c.p, E * 8, hipMemcpyDeviceToHost, c->stream));
        MD_TRY(sync(c));
        for (size_t e = 0; e < E; e++) {
            F.leaves[e].depth = (uint8_t)(key[e] & 15);
            for (int k = 0; k < 3; k++) F.leaves[e].c[k] = (uint32_t)((key[e] >> (4 + 20 * k)) & 0xfffff);
        }
    }
    F.face.clear();
    F.fine.clear();
    s->host_forest_valid = true;
    return MDLTS_OK;
}

mdlts_status alloc_canonical_state(mdlts_sim *s)
{
    const size_t n = (size_t)s->E * s->np * s->tsize;
    MD_TRY(dev_alloc(s->ctx, s->u_c, n));
    MD_TRY(dev_alloc(s->ctx, s->v_c, n));
    return MDLTS_OK;
}

mdlts_status zero_canonical_state(mdlts_sim *s)
{
    MD_TRY(alloc_canonical_state(s));
    const size_t n = (size_t)s->E * s->np * s->tsize;
    HIP_TRY(hipMemsetAsync(s->u_c.p, 0, n, s->ctx->stream));
    HIP_TRY(hipMemsetAsync(s->v_c.p, 0, n, s->ctx->stream));
    s->state_grouped = false;
    return MDLTS_OK;
}

// grouped -> canonical at a barrier
mdlts_status to_canonical(mdlts_sim *s, int *zero32 = nullptr)
{
    if (!s->state_grouped) return MDLTS_OK;
    const int E = (int)s->E;
    MD_TRY(alloc_canonical_state(s));
    const long long stride = (long long)s->np * s->cap;
    const int parity = (int)(s->n_since_assign & 1);
    if (s->desc.precision == MDLTS_FP64)
        k_gather<double><<<nblocks(E), kBlock, 0, s->ctx->stream>>>(E, s->np, s->cap, stride, P<int>(s->perm),
                                                                     P<int>(s->cnt_ge_d), parity, P<double>(s->u_s),
                                                                     P<double>(s->v_s), P<double>(s->u_c),
                                                                     P<double>(s->v_c), zero32);
    else
        k_gather<float><<<nblocks(E), kBlock, 0, s->ctx->stream>>>(E, s->np, s->cap, stride, P<int>(s->perm),
                                                                    P<int>(s->cnt_ge_d), parity, P<float>(s->u_s),
                                                                    P<float>(s->v_s), P<float>(s->u_c),
                                                                    P<float>(s->v_c), zero32);
    HIP_TRY(hipGetLastError());
    s->state_grouped = false;
    return MDLTS_OK;
}

// canonical -> grouped slot 0 (after a level assignment)
mdlts_status to_grouped(mdlts_sim *s)
{
    const int E = (int)s->E;
    if (s->desc.precision == MDLTS_FP64)
        k_permute<double><<<nblocks(E), kBlock, 0, s->ctx->stream>>>(E, s->np, s->cap, P<int>(s->perm),
                                                                      P<double>(s->u_c), P<double>(s->v_c),
                                                                      P<double>(s->u_s), P<double>(s->v_s));
    else
        k_permute<float><<<nblocks(E), kBlock, 0, s->ctx->stream>>>(E, s->np, s->cap, P<int>(s->perm),
                                                                     P<float>(s->u_c), P<float>(s->v_c),
                                                                     P<float>(s->u_s), P<float>(s->v_s));
    HIP_TRY(hipGetLastError());
    s->state_grouped = true;
    s->n_since_assign = 0;
    return MDLTS_OK;
}

mdlts_status set_forest(mdlts_sim *s, Forest &&F)
{
    s->tree_rev++;
    s->forest = std::move(F);
    s->levels_valid = false;
    s->eta_valid = false;
    return upload_forest(s);
}

// ---- substep launch -------------------------------------------------------
template <typename T>
mdlts_status launch_substep(const mdlts_sim *s, const StepArgs<T> *c, const StepLaunch<T> &L, hipStream_t st)
{
    void *fn = substep_kernel_of(kFormEager, s->desc.dim, s->desc.order, sizeof(T) == 4, s->dfull);
    if (!fn) return MDLTS_EINVAL;
    StepLaunch<T> Lv = L;
    void *args[] = {&c, &Lv};
    const size_t lds = gate_lds_bytes(s->desc.dim, s->desc.order, sizeof(T) == 4, kBlock);
    const long long threads = (long long)L.n_act * lanes_per_element(s->desc.dim, s->desc.order, s->dfull);
    HIP_TRY(hipLaunchKernel(fn, dim3(nblocks(threads)), dim3(kBlock), args, lds, st));
    return MDLTS_OK;
}

mdlts_status drain_events(mdlts_sim *s)
{
    if (s->ev_used == 0) return MDLTS_OK;
    HIP_TRY(hipEventSynchronize(s->ev[2 * s->ev_used - 1]));
    for (size_t q = 0; q < s->ev_used; q++) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, s->ev[2 * q], s->ev[2 * q + 1]));
        s->prof_ms += ms;
    }
    s->ev_used = 0;
    return MDLTS_OK;
}

constexpr size_t kMaxEventPairs = 4096;

// the per-assignment constants of the substep kernel, uploaded to the device
// when they change (parameters, levels, buffers)
template <typename T>
void fill_step_args(const mdlts_sim *s, StepArgs<T> &a)
{
    std::memset(&a, 0, sizeof(a));
    a.slot_stride = (long long)s->np * s->cap;
    a.slot_bytes = (uint32_t)(a.slot_stride * (long long)sizeof(T));
    a.node_bytes = (uint32_t)((long long)s->cap * (long long)sizeof(T));
    a.cap = s->cap;
    a.lmax = s->lmax;
    for (int l = 0; l < kMaxLevels; l++) a.cnt_ge[l] = l < (int)s->cnt_ge.size() && l <= s->lmax ? s->cnt_ge[l] : 0;
    a.dt_bar = s->dt_bar;
    for (int k = 0; k < 3; k++) {
        a.h0[k] = s->h0[k];
        a.inv_h0[k] = (T)(1.0 / s->h0[k]);
        a.Dk[k] = (T)s->Dk[k];
        a.Dx[k] = (T)s->Dx[k];
    }
    a.full = s->dfull ? 1 : 0;
    a.gamma = (T)s->gamma;
    a.apk = (T)s->ap.k;
    a.apa = (T)s->ap.a;
    a.eps0 = (T)s->ap.eps0;
    a.mu1 = (T)s->ap.mu1;
    a.mu2 = (T)s->ap.mu2;
    a.n_stim = (int)s->stim.size();
    for (int b = 0; b < a.n_stim; b++) {
        const mdlts_stim_box &x = s->stim[b];
        for (int k = 0; k < 3; k++) { a.stim[b][k] = x.lo[k]; a.stim[b][3 + k] = x.hi[k]; }
        a.stim[b][6] = x.t_on; a.stim[b][7] = x.t_off; a.stim[b][8] = x.amp;
    }
    fill_ref(s->ref, a.ref);
}

template <typename T>
mdlts_status upload_step_args(mdlts_sim *s)
{
    StepArgs<T> &a = *reinterpret_cast<StepArgs<T> *>(s->step_host.data());
    fill_step_args<T>(s, a);
    MD_TRY(dev_alloc(s->ctx, s->step_dev, sizeof(StepArgs<T>)));
    char *st = nullptr;
    MD_TRY(stage_acquire(s->ctx, sizeof(StepArgs<T>), &st));
    std::memcpy(st, &a, sizeof(StepArgs<T>));
    HIP_TRY(hipMemcpyAsync(s->step_dev.p, st, sizeof(StepArgs<T>), hipMemcpyHostToDevice, s->ctx->stream));
    MD_TRY(stage_release(s->ctx));
    s->step_dirty = false;
    return MDLTS_OK;
}

template <typename T>
mdlts_status run_barriers(mdlts_sim *s, int n_barriers)
{
    if (s->step_dirty) MD_TRY(upload_step_args<T>(s));
    StepLaunch<T> L;
    L.u = P<T>(s->u_s);
    L.v = P<T>(s->v_s);
    L.key = s->key_s.p;
    L.nbr = P<uint32_t>(s->nbr_s);
    L.fine = P<uint32_t>(s->fine_s);
    L.node_bytes = (uint32_t)((size_t)s->cap * sizeof(T));
    L.slot_bytes = (uint32_t)((size_t)s->np * s->cap * sizeof(T));
    L.cap = s->cap;
    L.lmax = s->lmax;
    const StepArgs<T> *cst = static_cast<const StepArgs<T> *>(s->step_dev.p);
    const long long maxS = 1ll << s->lmax;
    const double h_tick = s->dt_bar / (double)maxS;
    hipStream_t st = s->ctx->stream;
    for (int nb = 0; nb < n_barriers; nb++) {
        const double t_n = s->t_start + (double)s->n_bar * s->dt_bar;
        L.parity = (int)(s->n_since_assign & 1);
        for (long long i = 0; i < maxS; i++) {
            int v2 = 0;
            while (i > 0 && ((i >> v2) & 1) == 0) v2++;
            const int lmin = i == 0 ? 0 : s->lmax - v2;
            L.i = (int)i;
            L.n_act = s->cnt_ge[lmin];
            L.t_i = t_n + (double)i * h_tick;
            if (L.n_act == 0) continue;
            if (s->prof) {
                if (s->ev_used == kMaxEventPairs) MD_TRY(drain_events(s));
                while (s->ev.size() < 2 * (s->ev_used + 1)) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e));
                    s->ev.push_back(e);
                }
                HIP_TRY(hipEventRecord(s->ev[2 * s->ev_used], st));
            }
            MD_TRY(launch_substep<T>(s, cst, L, st));
            s->dof_updates += (uint64_t)L.n_act * (uint64_t)s->np;
            if (s->prof) {
                HIP_TRY(hipEventRecord(s->ev[2 * s->ev_used + 1], st));
                s->ev_used++;
                s->prof_launches++;
                s->prof_dof += (uint64_t)L.n_act * (uint64_t)s->np;
            }
        }
        HIP_TRY(hipGetLastError());
        s->n_bar++;
        s->n_since_assign++;
    }
    return MDLTS_OK;
}

template <int DIM, int P_, typename T>
void launch_indicator(const IndArgs &a, int E, hipStream_t st)
{
    if (a.full) k_indicator<DIM, P_, T, true><<<nblocks(E), kBlock, 0, st>>>(a);
    else k_indicator<DIM, P_, T, false><<<nblocks(E), kBlock, 0, st>>>(a);
}

// the indicator of the canonical state u (bulk precision, [np][E]) into eta
// [E], its maximum and non-finite flag into max_bits and nonfinite
template <typename T>
mdlts_status run_indicator(mdlts_sim *s, const void *u, double *eta, unsigned long long *max_bits, int *nonfinite)
{
    IndArgs a;
    std::memset(&a, 0, sizeof(a));
    const int E = (int)s->E;
    a.u = u;
    a.key = s->key_c.p;
    a.face = P<uint32_t>(s->face_c);
    a.fine = P<uint32_t>(s->fine_c);
    a.E = E;
    a.p = s->desc.order;
    for (int k = 0; k < 3; k++) { a.h0[k] = s->h0[k]; a.Dk[k] = s->Dk[k]; a.Dx[k] = s->Dx[k]; }
    a.full = s->dfull ? 1 : 0;
    fill_ref(s->ref, a.ref);
    a.eta = eta;
    a.eta_max_bits = max_bits;
    a.nonfinite = nonfinite;
    hipStream_t st = s->ctx->stream;
    switch (s->desc.dim * 10 + s->desc.order) {
    case 21: launch_indicator<2, 1, T>(a, E, st); break;
    case 22: launch_indicator<2, 2, T>(a, E, st); break;
    case 31: launch_indicator<3, 1, T>(a, E, st); break;
    case 32: launch_indicator<3, 2, T>(a, E, st); break;
    case 23: launch_indicator<2, 3, T>(a, E, st); break;
    case 33: launch_indicator<3, 3, T>(a, E, st); break;
    default: return MDLTS_EINVAL;
    }
    HIP_TRY(hipGetLastError());
    return MDLTS_OK;
}

// new canonical state from the old one through the device transfer map
// (xk: 0 copy, 1 prolong from the parent, 2 restrict from 2^d children)
template <typename T>
mdlts_status run_transfer(mdlts_sim *s, int E_old, int E_new)
{
    mdlts_ctx *c = s->ctx;
    const size_t bytes = (size_t)E_new * s->np * sizeof(T);
    MD_TRY(dev_alloc(c, s->tmp_u, bytes));
    MD_TRY(dev_alloc(c, s->tmp_v, bytes));
    XferArgs a;
    std::memset(&a, 0, sizeof(a));
    a.u_old = s->u_c.p;
    a.v_old = s->v_c.p;
    a.u_new = s->tmp_u.p;
    a.v_new = s->tmp_v.p;
    a.E_old = E_old;
    a.E_new = E_new;
    a.kind = P<uint8_t>(s->xk);
    a.src = P<int32_t>(s->xs);
    a.child = P<uint8_t>(s->xc);
    fill_ref(s->ref, a.ref);
    hipStream_t st = c->stream;
    switch (s->desc.dim * 10 + s->desc.order) {
    case 21: k_transfer<2, 1, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    case 22: k_transfer<2, 2, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    case 31: k_transfer<3, 1, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    case 32: k_transfer<3, 2, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    case 23: k_transfer<2, 3, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    case 33: k_transfer<3, 3, T><<<nblocks(E_new), kBlock, 0, st>>>(a); break;
    default: return MDLTS_EINVAL;
    }
    HIP_TRY(hipGetLastError());
    std::swap(s->u_c, s->tmp_u);
    std::swap(s->v_c, s->tmp_v);
    return MDLTS_OK;
}

// Algorithm 1's adaptation on the device, in two halves so that several
// simulations can share the synchronisation between them.
// First half: mark (eta >= tau_refine), close the 2:1 balance, flag
// coarsenable sibling groups, count and scan the new leaves; the counts
// arrive in pin->tallies / pin->total after the next synchronisation.
template <int DIM>
mdlts_status adapt_count(mdlts_sim *s, double tau_refine, double tau_coarsen, bool own_flags = true)
{
    using KT = typename KeyOf<DIM>::type;
    mdlts_ctx *c = s->ctx;
    hipStream_t st = c->stream;
    const int E = (int)s->E;
    const int nb = nblocks(E);
    const int nb4 = (E + 1023) / 1024;
    MD_TRY(dev_alloc(c, s->refine, (size_t)E));
    MD_TRY(dev_alloc(c, s->cflag, (size_t)E));
    MD_TRY(dev_alloc(c, s->cnt, (size_t)E * sizeof(int)));
    MD_TRY(dev_alloc(c, s->off, (size_t)E * sizeof(int)));
    MD_TRY(dev_alloc(c, s->bsums, (size_t)(nb4 + 1) * sizeof(int)));
    if (own_flags) MD_TRY(flags_clear(s));
    unsigned long long *tallies = MD_FLAG(s, unsigned long long, tallies);
    int *total = MD_FLAG(s, int, total);
    const MeshGeo g = geo_of(s);
    const KT *key = P<KT>(s->key_c);
    k_amr_mark<DIM><<<nb, kBlock, 0, st>>>(E, g, key, P<double>(s->eta_c), tau_refine, P<uint8_t>(s->refine));
    for (int pass = 0; pass < s->desc.max_depth; pass++)
        k_amr_close<DIM><<<nb, kBlock, 0, st>>>(E, P<uint32_t>(s->face_c), P<uint8_t>(s->refine));
    k_amr_coarsen<DIM><<<nb, kBlock, 0, st>>>(E, key, P<double>(s->eta_c), tau_coarsen, P<uint8_t>(s->refine),
                                               P<uint32_t>(s->face_c), P<uint8_t>(s->cflag));
    k_amr_count_scan<DIM><<<nb4, kBlock, 0, st>>>(E, key, P<uint8_t>(s->refine), P<uint8_t>(s->cflag), P<int>(s->cnt),
                                                   P<int>(s->off), P<int>(s->bsums), tallies);
    // block sums to block offsets and the total; the emit adds a leaf's
    // block offset to its block-local one
    k_scan_sums<<<1, kBlock, 0, st>>>(nb4, P<int>(s->bsums), total);
    HIP_TRY(hipGetLastError());
    // tallies and total are adjacent: one copy
    static_assert(offsetof(PinnedReadback, total) == 3 * sizeof(unsigned long long), "readback layout");
    if (own_flags)
        HIP_TRY(hipMemcpyAsync(s->pin->tallies, tallies, offsetof(PinnedReadback, total) + sizeof(int),
                               hipMemcpyDeviceToHost, st));
    return MDLTS_OK;
}

// Second half, after the counts are on the host: emit keys and the transfer
// map, transfer u and v, rebuild the face tables (their consistency flag
// arrives in pin->face_bad after the next synchronisation).
template <int DIM>
mdlts_status adapt_emit(mdlts_sim *s, bool own_flags = true)
{
    using KT = typename KeyOf<DIM>::type;
    mdlts_ctx *c = s->ctx;
    hipStream_t st = c->stream;
    const int E = (int)s->E;
    const int nb = nblocks(E);
    const int E_new = s->pin->total;
    if (E_new <= 0 || E_new >= (1 << 27)) return MDLTS_EINVAL;
    MD_TRY(dev_alloc(c, s->key_n, (size_t)E_new * sizeof(KT)));
    MD_TRY(dev_alloc(c, s->xk, (size_t)E_new));
    MD_TRY(dev_alloc(c, s->xs, (size_t)E_new * sizeof(int32_t)));
    MD_TRY(dev_alloc(c, s->xc, (size_t)E_new));
    k_amr_emit<DIM><<<nb, kBlock, 0, st>>>(E, P<KT>(s->key_c), P<uint8_t>(s->refine), P<uint8_t>(s->cflag),
                                            P<int>(s->cnt), P<int>(s->off), P<int>(s->bsums), P<KT>(s->key_n),
                                            P<uint8_t>(s->xk), P<int32_t>(s->xs), P<uint8_t>(s->xc));
    HIP_TRY(hipGetLastError());
    if (s->desc.precision == MDLTS_FP64) MD_TRY(run_transfer<double>(s, E, E_new));
    else MD_TRY(run_transfer<float>(s, E, E_new));
    std::swap(s->key_c, s->key_n);
    s->E = (size_t)E_new;
    s->tree_rev++;
    s->host_forest_valid = false;
    s->levels_valid = false;
    s->eta_valid = false;
    return device_faces(s, own_flags);
}

mdlts_status compute_G(mdlts_sim *s)
{
    if (!gershgorin_table(s->ref, s->gamma, s->G)) return MDLTS_EINVAL;
    return MDLTS_OK;
}


}  // namespace

// ---------------------------------------------------------------------------
// batches: many simulations advanced by one launch per substep and element
// kind; tile lists per substep; the barrier interval replayed as a hipGraph
// ---------------------------------------------------------------------------
struct BatchGroup {
    int dim = 2, order = 1, prec = 0;
    bool full = false;  // off-diagonal diffusion tensors (their own kernels)
    int block = 256;    // threads per block (= elements per tile), tuned per variant
    int variant_bit() const { return 12 * (full ? 1 : 0) + 6 * (dim - 2) + 2 * (order - 1) + (prec == MDLTS_FP32 ? 1 : 0); }
    std::vector<int> members;   // indices into BatchPlan::sims
    // one device buffer: descriptors [members] BatchSim, clocks [2][members]
    // BatchClock, tiles [2 phases][n_tiles] BatchTile (one upload)
    DevBuf data;
    size_t off_clocks = 0, off_tiles = 0;
    void *descs() const { return data.p; }
    BatchClock *clocks() const { return reinterpret_cast<BatchClock *>(static_cast<char *>(data.p) + off_clocks); }
    BatchTile *tiles() const { return reinterpret_cast<BatchTile *>(static_cast<char *>(data.p) + off_tiles); }
    std::vector<BatchClock> hclk;  // host source of the clock uploads
    // substep i launches tile_count[i] tiles from tile_start[i]; substeps
    // whose active sets are the same share one list
    std::vector<int> tile_start, tile_count;
    int n_tiles = 0;  // tiles in the distinct lists; the device holds two copies (phases)
    char *base = nullptr;
};

struct BatchPlan {
    std::vector<mdlts_sim *> sims;
    std::vector<uint64_t> versions;
    int lmax_all = 0;
    int block = 256;
    int per_cu = 0;  // always 0: one block per tile (reported by the profiling call)
    bool tuned = false;
    std::vector<BatchGroup> groups;
    std::vector<uint64_t> dof_per_barrier;  // per simulation
    std::vector<long long> n_bar;           // per simulation, as the device clocks hold it
    int variant_mask = 0;                   // kernel variants present
    int phase = 0;                          // clock copy the next barrier reads
    hipGraph_t graph[2] = {nullptr, nullptr};  // one barrier, per phase
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    // the graphs' kernel nodes in emission order and their keys (substep,
    // kernel variant); a plan whose launches have the same keys updates the
    // nodes' parameters instead of building new graphs
    std::vector<hipGraphNode_t> nodes[2];
    std::vector<long long> topo;
    bool graph_valid = false;  // the graphs hold this plan's current launches
    bool graph_busy = false;   // a replay was launched in sync epoch busy_epoch
    uint64_t busy_epoch = 0;
    bool single_graph = false;  // a one-variant plan replays graphs (tuned)
    // optional event timing of every batched substep launch
    bool prof = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double prof_ms = 0.0;
    uint64_t prof_launches = 0, prof_dof = 0;
};

namespace {

void destroy_graph(BatchPlan *P)
{
    for (int k = 0; k < 2; k++) {
        if (P->exec[k]) (void)hipGraphExecDestroy(P->exec[k]);
        if (P->graph[k]) (void)hipGraphDestroy(P->graph[k]);
        P->exec[k] = nullptr;
        P->graph[k] = nullptr;
        P->nodes[k].clear();
    }
    P->topo.clear();
    P->graph_valid = false;
}

// the plan's launches changed: its graphs must be updated or rebuilt before
// the next replay
void free_graph(BatchPlan *P) { P->graph_valid = false; }

// hands the graphs of `from` (a plan being replaced) to `to`, for reuse
void adopt_graph(BatchPlan *to, BatchPlan *from)
{
    if (!from || !to) return;
    for (int k = 0; k < 2; k++) {
        to->graph[k] = from->graph[k];
        to->exec[k] = from->exec[k];
        to->nodes[k].swap(from->nodes[k]);
        from->graph[k] = nullptr;
        from->exec[k] = nullptr;
    }
    to->topo.swap(from->topo);
    to->graph_valid = false;
    to->graph_busy = from->graph_busy;
    to->busy_epoch = from->busy_epoch;
}

// frees a plan (the context's batch plan or a simulation's step plan)
// (sync_first = false: the plan's graphs have been handed over and its
// buffers are freed in stream order: through the allocator, or by hipFree,
// which waits for the device)
void free_plan(mdlts_ctx *c, BatchPlan *&slot, bool sync_first = true)
{
    BatchPlan *P = slot;
    if (!P) return;
    if (sync_first) (void)hipStreamSynchronize(c->stream);
    destroy_graph(P);
    for (auto &g : P->groups) {
        dev_free(c, g.data);
    }
    for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
    delete P;
    slot = nullptr;
}

void *batch_kernel(int dim, int order, int prec, bool full)
{
    return substep_kernel_of(kFormBatch, dim, order, prec == MDLTS_FP32, full);
}


// A run of tiles of one simulation and level in a tile list: tiles k0 ..
// k0 + n - 1 cover elements [lo, hi) in pieces of per_tile; t holds the
// fields they share (the parity of the list's barrier in t.packed).  The
// host sends the runs; k_expand_tiles writes the tiles on the device.
struct TileRun {
    BatchTile t;
    int k0, n, lo, hi, per_tile;
    int pad[3];
};
static_assert(sizeof(TileRun) == 96, "tile runs pack without holes");

// tile k of a list of n_tiles from its runs (ascending k0), into the list of
// this barrier's parity (t0) and of the next one's (t1)
__global__ __launch_bounds__(256) void k_expand_tiles(const TileRun *__restrict__ runs, int n_runs,
                                                      BatchTile *__restrict__ t0, BatchTile *__restrict__ t1,
                                                      int n_tiles)
{
    const int k = (int)(blockIdx.x * 256 + threadIdx.x);
    if (k >= n_tiles) return;
    int lo = 0, hi = n_runs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (runs[mid].k0 <= k) lo = mid;
        else hi = mid - 1;
    }
    const TileRun &r = runs[lo];
    BatchTile tt = r.t;
    tt.start = r.lo + (k - r.k0) * r.per_tile;
    tt.count = min(r.per_tile, r.hi - tt.start);
    t0[k] = tt;
    tt.packed ^= 1 << 4;
    t1[k] = tt;
}

template <typename T>
mdlts_status fill_group(mdlts_ctx *c, BatchPlan &P, BatchGroup &G)
{
    const int nm = (int)G.members.size();
    const int per_tile = elements_per_block(G.dim, G.order, G.full, G.block);  // elements per tile
    // tile lists: substep i of the barrier interval (each simulation runs
    // its own 2^lmax substeps; shorter schedules idle at the end).  Active
    // levels lmax..lmin of a simulation occupy [0, cnt_ge[lmin]), finest
    // first, and tiles do not straddle levels.  The tiles are counted first
    // and then written straight into the pinned staging area.
    const long long nsub = 1ll << P.lmax_all;
    auto lmin_of = [](long long i, int lmax) {
        int v2 = 0;
        while (i > 0 && ((i >> v2) & 1) == 0) v2++;
        return i == 0 ? 0 : lmax - v2;
    };
    auto level_range = [](const mdlts_sim *s, int l, int &lo, int &hi) {
        lo = l == s->lmax ? 0 : s->cnt_ge[l + 1];
        hi = s->cnt_ge[l];
    };
    // a substep's list is fixed by each member's lowest active level (-1:
    // past the member's schedule); the distinct lists are kept once each
    std::map<std::vector<int>, int> seen;  // active levels -> list
    std::vector<long long> first;          // first substep of each list
    G.tile_start.assign(nsub, 0);
    G.tile_count.assign(nsub, 0);
    size_t nt = 0;
    std::vector<int> sig(nm);
    for (long long i = 0; i < nsub; i++) {
        for (int q = 0; q < nm; q++) {
            const mdlts_sim *s = P.sims[G.members[q]];
            sig[q] = i < (1ll << s->lmax) ? lmin_of(i, s->lmax) : -1;
        }
        auto it = seen.find(sig);
        if (it != seen.end()) {
            G.tile_start[i] = G.tile_start[first[it->second]];
            G.tile_count[i] = G.tile_count[first[it->second]];
            continue;
        }
        seen.emplace(sig, (int)first.size());
        first.push_back(i);
        size_t n_i = 0;
        for (int q = 0; q < nm; q++) {
            if (sig[q] < 0) continue;
            const mdlts_sim *s = P.sims[G.members[q]];
            for (int l = s->lmax; l >= sig[q]; l--) {
                int lo, hi;
                level_range(s, l, lo, hi);
                if (hi > lo) n_i += (size_t)((hi - lo + per_tile - 1) / per_tile);
            }
        }
        G.tile_start[i] = (int)nt;
        G.tile_count[i] = (int)n_i;
        nt += n_i;
    }
    G.n_tiles = (int)nt;
    // descriptors, clocks, the runs and both tile lists (this barrier's
    // parity and the next one's) in one buffer; the host sends descriptors,
    // clocks and runs in one copy and the device writes the tiles
    size_t n_runs = 0;
    for (const long long i : first)
        for (int q = 0; q < nm; q++) {
            const mdlts_sim *s = P.sims[G.members[q]];
            if (i >= (1ll << s->lmax)) continue;
            for (int l = s->lmax; l >= lmin_of(i, s->lmax); l--) {
                int lo, hi;
                level_range(s, l, lo, hi);
                if (hi > lo) n_runs++;
            }
        }
    const size_t b_d = (size_t)nm * sizeof(BatchSim<T>), b_c = 2 * (size_t)nm * sizeof(BatchClock);
    const size_t b_r = n_runs * sizeof(TileRun);
    const size_t b_t = 2 * nt * sizeof(BatchTile);
    G.off_clocks = (b_d + 255) / 256 * 256;
    const size_t off_runs = G.off_clocks + (b_c + 255) / 256 * 256;
    G.off_tiles = off_runs + (b_r + 255) / 256 * 256;
    const size_t total = G.off_tiles + std::max<size_t>(b_t, sizeof(BatchTile));
    MD_TRY(dev_alloc(c, G.data, total));
    G.base = static_cast<char *>(G.data.p);
    char *st = nullptr;
    MD_TRY(stage_acquire(c, G.off_tiles, &st));
    for (int q = 0; q < nm; q++) {
        mdlts_sim *s = P.sims[G.members[q]];
        BatchSim<T> d;
        std::memset(&d, 0, sizeof(d));
        fill_step_args<T>(s, d.a);
        d.t_start = s->t_start;
        d.h_tick = s->dt_bar / (double)(1ll << s->lmax);
        std::memcpy(st + (size_t)q * sizeof(BatchSim<T>), &d, sizeof(d));
    }
    G.hclk.resize(2 * (size_t)nm);
    for (int q = 0; q < nm; q++) G.hclk[q] = G.hclk[nm + q] = BatchClock{P.sims[G.members[q]]->n_bar};
    std::memcpy(st + G.off_clocks, G.hclk.data(), b_c);
    TileRun *rr = reinterpret_cast<TileRun *>(st + off_runs);
    size_t k = 0, r = 0;
    const long long dbase = (long long)(uintptr_t)G.base;
    for (const long long i : first)
        for (int q = 0; q < nm; q++) {
            const mdlts_sim *s = P.sims[G.members[q]];
            if (i >= (1ll << s->lmax)) continue;
            TileRun run;
            std::memset(&run, 0, sizeof(run));
            BatchTile &tt = run.t;  // array locations as offsets from the buffer's base
            tt.off_u = (long long)(uintptr_t)s->u_s.p - dbase;
            tt.off_v = (long long)(uintptr_t)s->v_s.p - dbase;
            tt.off_key = (long long)(uintptr_t)s->key_s.p - dbase;
            tt.off_nbr = (long long)(uintptr_t)s->nbr_s.p - dbase;
            tt.off_fine = (long long)(uintptr_t)s->fine_s.p - dbase;
            tt.sim = q;
            tt.node_bytes = (uint32_t)((size_t)s->cap * sizeof(T));
            tt.slot_bytes = (uint32_t)((size_t)s->np * s->cap * sizeof(T));
            const int parity = (int)(s->n_since_assign & 1);
            for (int l = s->lmax; l >= lmin_of(i, s->lmax); l--) {
                int lo, hi;
                level_range(s, l, lo, hi);
                if (hi <= lo) continue;
                tt.packed = l | parity << 4 | s->lmax << 8;
                run.k0 = (int)k;
                run.n = (hi - lo + per_tile - 1) / per_tile;
                run.lo = lo;
                run.hi = hi;
                run.per_tile = per_tile;
                if (r >= n_runs) return MDLTS_EINVAL;
                std::memcpy(rr + r, &run, sizeof(run));
                r++;
                k += (size_t)run.n;
            }
        }
    if (k != nt || r != n_runs) return MDLTS_EINVAL;  // the passes disagree (cannot happen)
    HIP_TRY(hipMemcpyAsync(G.data.p, st, G.off_tiles, hipMemcpyHostToDevice, c->stream));
    if (nt > 0) {
        BatchTile *dt0 = G.tiles();
        k_expand_tiles<<<(unsigned)((nt + 255) / 256), 256, 0, c->stream>>>(
            reinterpret_cast<const TileRun *>(G.base + off_runs), (int)n_runs, dt0, dt0 + nt, (int)nt);
        HIP_TRY(hipGetLastError());
    }
    return stage_release(c);
}

// (re)build descriptors and tile lists for the current launch shape
mdlts_status build_plan_data(mdlts_ctx *c, BatchPlan &P)
{
    free_graph(&P);
    for (auto &G : P.groups)
        MD_TRY(G.prec == MDLTS_FP64 ? fill_group<double>(c, P, G) : fill_group<float>(c, P, G));
    P.phase = 0;
    P.n_bar.resize(P.sims.size());
    for (size_t q = 0; q < P.sims.size(); q++) P.n_bar[q] = P.sims[q]->n_bar;
    return MDLTS_OK;
}

// one block per tile: 8 times the largest XCD share (tiles are dealt to the
// XCDs in contiguous ranges)
int grid_of(const BatchPlan &P, int n_tiles)
{
    (void)P;
    return std::max((n_tiles + 7) / 8 * 8, 8);
}

// one barrier interval reading clock copy `phase`: launches on the stream,
// or kernel nodes of a graph.  In a graph each kernel variant's launches
// form a chain of their own (substep after substep): the variants hold
// disjoint simulations, so one variant's later substeps overlap another's
// longer launches.
enum EmitMode { kEmitLaunch, kEmitGraph, kEmitUpdate, kEmitKeys };

// Where kEmitGraph puts a barrier's nodes and which nodes kEmitUpdate sets:
// consecutive barriers emitted into one target form one graph, each
// group's chain continuing from one barrier into the next.
struct GraphTarget {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> *nodes = nullptr;  // in emission order
    std::vector<hipGraphNode_t> last;              // per group: its latest node
    size_t n_node = 0;                             // next node to update
};

mdlts_status emit_barrier(mdlts_ctx *c, BatchPlan &P, int phase, GraphTarget *gt, EmitMode mode = kEmitLaunch,
                          std::vector<long long> *keys = nullptr, std::vector<hipEvent_t> *timed = nullptr,
                          std::vector<int> *timed_group = nullptr)
{
    // timed (direct launches only): an event pair around every launch, and
    // the index of the launch's group in timed_group
    if ((mode == kEmitGraph || mode == kEmitUpdate) && (!gt || !gt->nodes)) return MDLTS_EINVAL;
    if (mode != kEmitLaunch) timed = nullptr;
    if (gt) gt->last.resize(P.groups.size(), nullptr);
    size_t n_timed = 0;
    const long long nsub = 1ll << P.lmax_all;
    auto add = [&](long long key, size_t g, void *fn, int grid, int block, size_t lds, void **args) -> mdlts_status {
        hipKernelNodeParams kp{};
        kp.func = fn;
        kp.gridDim = dim3(grid);
        kp.blockDim = dim3(block);
        kp.sharedMemBytes = (unsigned int)lds;
        kp.kernelParams = args;
        kp.extra = nullptr;
        if (mode == kEmitGraph) {
            hipGraphNode_t node;
            hipGraphNode_t *dep = gt->last[g] ? &gt->last[g] : nullptr;
            HIP_TRY(hipGraphAddKernelNode(&node, gt->graph, dep, dep ? 1 : 0, &kp));
            gt->last[g] = node;
            gt->nodes->push_back(node);
            if (keys) keys->push_back(key);
        } else if (mode == kEmitUpdate) {
            if (gt->n_node >= gt->nodes->size()) return MDLTS_EINVAL;
            HIP_TRY(hipGraphExecKernelNodeSetParams(gt->exec, (*gt->nodes)[gt->n_node++], &kp));
        } else if (mode == kEmitKeys) {
            keys->push_back(key);
        } else {
            HIP_TRY(hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, c->stream));
        }
        return MDLTS_OK;
    };
    for (long long i = 0; i < nsub; i++) {
        for (auto &G : P.groups) {
            int n_t = G.tile_count[i];
            if (n_t == 0) continue;
            const void *descs = G.descs();
            const BatchTile *tl = G.tiles() + (size_t)phase * G.n_tiles + G.tile_start[i];
            int ii = (int)i;
            char *base = G.base;
            const int nm = (int)G.members.size();
            const BatchClock *ck = G.clocks() + (size_t)phase * nm;
            BatchClock *ck_next = G.clocks() + (size_t)(phase ^ 1) * nm;
            void *args[] = {&descs, &tl, &n_t, &ii, &base, &ck, &ck_next};
            const bool prof = P.prof && mode == kEmitLaunch;
            if (prof) {
                while (P.ev.size() < 2 * (P.ev_used + 1)) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e));
                    P.ev.push_back(e);
                }
                HIP_TRY(hipEventRecord(P.ev[2 * P.ev_used], c->stream));
            }
            const long long key = i * 64 + 12 * (G.full ? 1 : 0) + 6 * (G.dim - 2) + 2 * (G.order - 1) +
                                  (G.prec == MDLTS_FP32 ? 1 : 0);
            if (timed) {
                while (timed->size() < 2 * (n_timed + 1)) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e));
                    timed->push_back(e);
                }
                HIP_TRY(hipEventRecord((*timed)[2 * n_timed], c->stream));
            }
            const size_t g = (size_t)(&G - P.groups.data());
            MD_TRY(add(key, g, batch_kernel(G.dim, G.order, G.prec, G.full), grid_of(P, n_t), G.block,
                       gate_lds_bytes(G.dim, G.order, G.prec == MDLTS_FP32, G.block), args));
            if (timed) {
                HIP_TRY(hipEventRecord((*timed)[2 * n_timed + 1], c->stream));
                if (timed_group) timed_group->push_back((int)g);
                n_timed++;
            }
            if (prof) {
                HIP_TRY(hipEventRecord(P.ev[2 * P.ev_used + 1], c->stream));
                P.ev_used++;
                P.prof_launches++;
            }
        }
    }
    return MDLTS_OK;
}

// Barriers per graph (even: a graph ends on the clock copy it starts with):
// more for plans of several kernel variants, whose chains overlap across
// the barriers inside a graph; a one-variant plan is a single chain.
int graph_barriers(const BatchPlan &P) { return P.groups.size() > 1 ? 8 : 4; }

// The graphs of the plan's current launches, graph_barriers(P) barriers each
// (graph k starts with clock copy k): the nodes of graphs already built for
// the same keys get the new parameters (grids, blocks, tile lists, clocks);
// otherwise the graphs are built anew.
mdlts_status build_graph(mdlts_ctx *c, BatchPlan &P)
{
    if (P.exec[0] && P.exec[1]) {
        std::vector<long long> keys;
        MD_TRY(emit_barrier(c, P, 0, nullptr, kEmitKeys, &keys));
        const size_t n = (size_t)graph_barriers(P) * keys.size();
        if (keys == P.topo && P.nodes[0].size() == n && P.nodes[1].size() == n) {
            // no replay of these graphs may be in flight while they change
            // (a stream synchronisation since the last replay suffices)
            if (P.graph_busy && P.busy_epoch == c->sync_epoch) MD_TRY(sync(c));
            P.graph_busy = false;
            for (int k = 0; k < 2; k++) {
                GraphTarget gt;
                gt.exec = P.exec[k];
                gt.nodes = &P.nodes[k];
                for (int h = 0; h < graph_barriers(P); h++) MD_TRY(emit_barrier(c, P, k ^ (h & 1), &gt, kEmitUpdate));
            }
            P.graph_valid = true;
            return MDLTS_OK;
        }
    }
    destroy_graph(&P);
    for (int k = 0; k < 2; k++) {
        HIP_TRY(hipGraphCreate(&P.graph[k], 0));
        GraphTarget gt;
        gt.graph = P.graph[k];
        gt.nodes = &P.nodes[k];
        std::vector<long long> keys;
        MD_TRY(emit_barrier(c, P, k, &gt, kEmitGraph, &keys));
        for (int h = 1; h < graph_barriers(P); h++) MD_TRY(emit_barrier(c, P, k ^ (h & 1), &gt, kEmitGraph));
        HIP_TRY(hipGraphInstantiate(&P.exec[k], P.graph[k], nullptr, nullptr, 0));
        if (k == 0) P.topo = keys;
    }
    P.graph_valid = true;
    return MDLTS_OK;
}

// host-side bookkeeping of nb barriers run by the batch (the clock copies
// alternate, so an odd count changes the phase)
void account_barriers(BatchPlan &P, int nb)
{
    for (size_t q = 0; q < P.sims.size(); q++) {
        mdlts_sim *s = P.sims[q];
        s->n_bar += nb;
        s->n_since_assign += nb;
        s->dof_updates += P.dof_per_barrier[q] * (uint64_t)nb;
        s->eta_valid = false;
        P.n_bar[q] = s->n_bar;
    }
    P.phase ^= nb & 1;
    if (P.prof)
        for (size_t q = 0; q < P.sims.size(); q++) P.prof_dof += P.dof_per_barrier[q] * (uint64_t)nb;
}

mdlts_status drain_batch_events(BatchPlan &P)
{
    if (P.ev_used == 0) return MDLTS_OK;
    HIP_TRY(hipEventSynchronize(P.ev[2 * P.ev_used - 1]));
    for (size_t q = 0; q < P.ev_used; q++) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, P.ev[2 * q], P.ev[2 * q + 1]));
        P.prof_ms += ms;
    }
    P.ev_used = 0;
    return MDLTS_OK;
}

mdlts_status run_batch_barriers(mdlts_ctx *c, BatchPlan &P, int nb)
{
    const bool graphs = c->use_graphs && (P.groups.size() > 1 || P.single_graph) && !P.prof;
    int b = 0;
    while (b < nb) {
        const int gb = graph_barriers(P);
        if (graphs && nb - b >= gb) {
            // gb barriers per graph; each kernel variant's
            // launches are a chain of their own through all of them, and
            // the chains run concurrently.  A plan of one variant (a single
            // chain) replays graphs only if the autotuner found them faster
            // than direct launches; the barriers of a call that do not fill
            // a graph are launched directly.
            if (!P.graph_valid) MD_TRY(build_graph(c, P));
            HIP_TRY(hipGraphLaunch(P.exec[P.phase], c->stream));
            P.graph_busy = true;
            P.busy_epoch = c->sync_epoch;
            account_barriers(P, gb);
            b += gb;
            continue;
        }
        if (P.prof && P.ev_used + P.groups.size() * (1u << P.lmax_all) > kMaxEventPairs)
            MD_TRY(drain_batch_events(P));
        MD_TRY(emit_barrier(c, P, P.phase, nullptr));
        account_barriers(P, 1);
        b++;
    }
    return MDLTS_OK;
}

// the tuned launch shapes of a plan's mix of kernel variants
void ctx_tuned_store(mdlts_ctx *c, const BatchPlan &P, double dof)
{
    mdlts_ctx::Tuned t;
    for (const BatchGroup &G : P.groups) t.blocks[G.variant_bit()] = G.block;
    t.block = P.block;
    t.dof = dof;
    t.single_graph = P.single_graph;
    c->tuned[P.variant_mask] = t;
}

// Autotuner: the first barriers of a new plan are run with each candidate
// block size (threads per block = elements per tile; one block per tile),
// the same for every kernel variant, in rounds over the candidates, with an
// event pair around every launch (one warm and one timed barrier per
// candidate and round).  Each variant keeps the candidate with its smallest
// launch time summed over the barrier, taking the best round: the variants
// differ (small elements favour small blocks, 27-node hexahedra large
// ones).  A one-variant plan then times graph replay of its shape against
// its direct launches.  Per-element arithmetic does not depend on the
// choice, so results are unchanged.
mdlts_status autotune(mdlts_ctx *c, BatchPlan &P, int *remaining)
{
    const int cands[] = {256, 128, 64};
    constexpr int n_cand = (int)(sizeof(cands) / sizeof(cands[0]));
    constexpr int rounds = 2;
    if (*remaining < n_cand * rounds * 2) return MDLTS_OK;
    struct Events {  // destroyed on every return
        std::vector<hipEvent_t> v;
        ~Events()
        {
            for (hipEvent_t e : v) (void)hipEventDestroy(e);
        }
    } tev, pair;
    pair.v.resize(2, nullptr);
    HIP_TRY(hipEventCreate(&pair.v[0]));
    HIP_TRY(hipEventCreate(&pair.v[1]));
    hipEvent_t e0 = pair.v[0], e1 = pair.v[1];
    const size_t ng = P.groups.size();
    std::vector<double> best(ng * n_cand, 1e300);
    std::vector<int> tgrp;
    const bool saved_prof = P.prof;
    P.prof = false;
    for (int rd = 0; rd < rounds; rd++)
        for (int k = 0; k < n_cand; k++) {
            for (BatchGroup &G : P.groups) G.block = cands[k];
            MD_TRY(build_plan_data(c, P));
            MD_TRY(emit_barrier(c, P, P.phase, nullptr));  // warm
            account_barriers(P, 1);
            tgrp.clear();
            MD_TRY(emit_barrier(c, P, P.phase, nullptr, kEmitLaunch, nullptr, &tev.v, &tgrp));
            account_barriers(P, 1);
            *remaining -= 2;
            if (tgrp.empty()) continue;
            HIP_TRY(hipEventSynchronize(tev.v[2 * tgrp.size() - 1]));
            std::vector<double> sum(ng, 0.0);
            for (size_t n = 0; n < tgrp.size(); n++) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, tev.v[2 * n], tev.v[2 * n + 1]));
                sum[tgrp[n]] += ms;
            }
            for (size_t g = 0; g < ng; g++) best[g * n_cand + k] = std::min(best[g * n_cand + k], sum[g]);
        }
    // each variant its fastest candidate; the plan reports the block size
    // of the variant with the most device time
    double top = -1.0;
    for (size_t g = 0; g < ng; g++) {
        int pick = 0;
        for (int k = 1; k < n_cand; k++)
            if (best[g * n_cand + k] < best[g * n_cand + pick]) pick = k;
        P.groups[g].block = cands[pick];
        if (best[g * n_cand + pick] > top) {
            top = best[g * n_cand + pick];
            P.block = cands[pick];
        }
    }
    // one kernel variant: graph replay against direct launches of the
    // chosen shape, each over a run of barriers (the host runs ahead of the
    // device in both; long chains of short launches favour the graph, a
    // few longer ones the direct launches, whose host cost is lower)
    P.single_graph = false;
    constexpr int runs = 1;  // timed graph-sized runs of barriers after one warm run
    const int gb = graph_barriers(P);
    if (c->use_graphs && P.groups.size() == 1 && *remaining >= 2 * gb * (runs + 1)) {
        MD_TRY(build_plan_data(c, P));
        float t_direct = 0.f, t_graph = 0.f;
        for (int mode = 0; mode < 2; mode++) {
            if (mode == 1) MD_TRY(build_graph(c, P));
            for (int b = 0; b <= runs; b++) {
                if (b == 1) HIP_TRY(hipEventRecord(e0, c->stream));
                if (mode == 1) {
                    HIP_TRY(hipGraphLaunch(P.exec[P.phase], c->stream));
                    P.graph_busy = true;
                    P.busy_epoch = c->sync_epoch;
                    account_barriers(P, gb);
                } else {
                    for (int h = 0; h < gb; h++) {
                        MD_TRY(emit_barrier(c, P, P.phase, nullptr));
                        account_barriers(P, 1);
                    }
                }
            }
            HIP_TRY(hipEventRecord(e1, c->stream));
            HIP_TRY(hipEventSynchronize(e1));
            P.graph_busy = false;
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            (mode == 1 ? t_graph : t_direct) = ms;
            *remaining -= gb * (runs + 1);
        }
        P.single_graph = t_graph < t_direct;
    }
    P.prof = saved_prof;
    P.tuned = true;
    double dof = 0.0;
    for (uint64_t d : P.dof_per_barrier) dof += (double)d;
    ctx_tuned_store(c, P, dof);
    return build_plan_data(c, P);
}

// The plan in `slot` for these simulations, rebuilt when the set or any
// simulation's levels, buffers or parameters changed; when only barrier
// counts moved (the simulations were stepped by another plan) the clocks
// are uploaded again.
mdlts_status prepare_plan(mdlts_ctx *c, BatchPlan *&slot, mdlts_sim *const *sims, int n, bool *fresh)
{
    *fresh = false;
    BatchPlan *P = slot;
    bool same = P && (int)P->sims.size() == n;
    for (int q = 0; same && q < n; q++) same = P->sims[q] == sims[q] && P->versions[q] == sims[q]->version;
    if (same) {
        bool moved = false;
        for (int q = 0; q < n; q++) moved = moved || P->n_bar[q] != sims[q]->n_bar;
        // clocks and the tiles' parities from the host's counts
        if (moved) MD_TRY(build_plan_data(c, *P));
        return MDLTS_OK;
    }
    // the replaced plan is freed on every way out, after its graphs and
    // device buffers have been handed over
    struct OldPlan {
        mdlts_ctx *c;
        BatchPlan *p;
        ~OldPlan() { free_plan(c, p, false); }
    } old{c, slot};
    P = new (std::nothrow) BatchPlan;
    if (!P) return MDLTS_ENOMEM;
    adopt_graph(P, old.p);  // the replaced plan's graphs, for a parameter update
    slot = P;
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];  // (its step constants travel in the plan's descriptors)
        P->sims.push_back(s);
        P->lmax_all = std::max(P->lmax_all, s->lmax);
        uint64_t dof = 0;
        for (long long i = 0; i < (1ll << s->lmax); i++) {
            int v2 = 0;
            while (i > 0 && ((i >> v2) & 1) == 0) v2++;
            dof += (uint64_t)s->cnt_ge[i == 0 ? 0 : s->lmax - v2] * (uint64_t)s->np;
        }
        P->dof_per_barrier.push_back(dof);
        int g = -1;
        for (size_t k = 0; k < P->groups.size(); k++)
            if (P->groups[k].dim == s->desc.dim && P->groups[k].order == s->desc.order &&
                P->groups[k].prec == s->desc.precision && P->groups[k].full == s->dfull)
                g = (int)k;
        if (g < 0) {
            P->groups.emplace_back();
            g = (int)P->groups.size() - 1;
            P->groups[g].dim = s->desc.dim;
            P->groups[g].order = s->desc.order;
            P->groups[g].prec = s->desc.precision;
            P->groups[g].full = s->dfull;
        }
        P->groups[g].members.push_back(q);
    }
    for (int q = 0; q < n; q++) P->versions.push_back(sims[q]->version);
    // groups of a kernel variant the replaced plan had take over its device
    // buffers (descriptors, tiles, clocks): no allocator round trips
    if (old.p)
        for (BatchGroup &G : P->groups)
            for (BatchGroup &O : old.p->groups)
                if (O.dim == G.dim && O.order == G.order && O.prec == G.prec && O.full == G.full && O.data.p) {
                    std::swap(G.data, O.data);
                    break;
                }
    for (const BatchGroup &g : P->groups) P->variant_mask |= 1 << g.variant_bit();
    // a mix of variants tuned before keeps its launch shape while the work
    // per barrier stays within 25 % of what it was tuned on (the best shape
    // moves as meshes refine)
    const auto tk = c->tuned.find(P->variant_mask);
    double dof = 0.0;
    for (uint64_t d : P->dof_per_barrier) dof += (double)d;
    if (tk != c->tuned.end() && std::fabs(dof - tk->second.dof) <= 0.25 * tk->second.dof) {
        for (BatchGroup &G : P->groups) {
            const auto b = tk->second.blocks.find(G.variant_bit());
            G.block = b != tk->second.blocks.end() ? b->second : tk->second.block;
        }
        P->block = tk->second.block;
        P->single_graph = tk->second.single_graph;
        P->tuned = true;
    }
    *fresh = true;
    return build_plan_data(c, *P);
}

// ---------------------------------------------------------------------------
// adaptation of many simulations with one launch per step and kernel variant
// ---------------------------------------------------------------------------
// a simulation's flags block: cleared, or copied to its row of the
// collection buffer (one block each)
struct ClearFlagsOp {
    int *flags;
    __device__ __forceinline__ void operator()(const int) const
    {
        if (threadIdx.x < kFlagBytes / sizeof(int)) flags[threadIdx.x] = 0;
    }
};
struct CopyFlagsOp {
    const int *flags;
    int *row;
    __device__ __forceinline__ void operator()(const int) const
    {
        if (threadIdx.x < kFlagBytes / sizeof(int)) row[threadIdx.x] = flags[threadIdx.x];
    }
};

// The launches of one phase over many simulations.  Ops added between two
// step() calls form one step: one k_multi launch per op type (kernel
// variant), which the simulations' data keep independent; the steps run in
// order on the context stream.  run() sends every op table of the phase to
// the device in one copy before the first launch.
class MultiPhase {
    struct AnyBatch {
        virtual ~AnyBatch() = default;
        virtual void emit(MultiPhase &m) = 0;
    };
    template <typename Op>
    struct TypedBatch : AnyBatch {
        std::vector<Op> ops;
        std::vector<int> block0;
        long long total = 0;
        void emit(MultiPhase &m) override { m.emit_launch(ops, block0, total); }
    };
    template <typename Op>
    static const void *tag()
    {
        static const char t = 0;
        return &t;
    }
    std::vector<std::pair<const void *, std::unique_ptr<AnyBatch>>> cur_;
    std::vector<char> table_;
    std::vector<std::function<void(hipStream_t, char *)>> steps_;

    size_t put(const void *p, size_t bytes)
    {
        const size_t off = (table_.size() + 15) & ~(size_t)15;
        table_.resize(off + bytes);
        std::memcpy(table_.data() + off, p, bytes);
        return off;
    }
    template <typename Op>
    void emit_launch(const std::vector<Op> &ops, const std::vector<int> &block0, long long total)
    {
        const size_t o_ops = put(ops.data(), ops.size() * sizeof(Op));
        const size_t o_b0 = put(block0.data(), block0.size() * sizeof(int));
        const int n = (int)ops.size();
        const unsigned grid = (unsigned)total;
        steps_.push_back([=](hipStream_t st, char *dev) {
            k_multi<Op><<<grid, kBlock, 0, st>>>(reinterpret_cast<const Op *>(dev + o_ops),
                                                 reinterpret_cast<const int *>(dev + o_b0), n);
        });
    }

public:
    template <typename Op>
    void add(const Op &op, long long n_blocks)
    {
        if (n_blocks <= 0) return;
        TypedBatch<Op> *t = nullptr;
        for (auto &e : cur_)
            if (e.first == tag<Op>()) t = static_cast<TypedBatch<Op> *>(e.second.get());
        if (!t) {
            auto u = std::make_unique<TypedBatch<Op>>();
            t = u.get();
            cur_.emplace_back(tag<Op>(), std::move(u));
        }
        t->ops.push_back(op);
        t->block0.push_back((int)t->total);
        t->total += n_blocks;
    }
    void step()
    {
        for (auto &e : cur_) e.second->emit(*this);
        cur_.clear();
    }
    // work other than launches (copies), in order after the steps so far
    void then(std::function<void(hipStream_t, char *)> f)
    {
        step();
        steps_.push_back(std::move(f));
    }
    mdlts_status run(mdlts_ctx *c)
    {
        step();
        if (steps_.empty()) return MDLTS_OK;
        const size_t bytes = std::max(table_.size(), (size_t)16);
        // the staging area is free: every copy out of it precedes the
        // synchronisation that ended the previous phase
        if (c->multi_host_bytes < bytes) {
            if (c->multi_host) (void)hipHostFree(c->multi_host);
            c->multi_host = nullptr;
            c->multi_host_bytes = 0;
            const size_t nb = std::max(bytes + bytes / 4, (size_t)64 << 10);
            if (hipHostMalloc(&c->multi_host, nb, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                c->multi_host = nullptr;
                return MDLTS_ENOMEM;
            }
            c->multi_host_bytes = nb;
        }
        if (!table_.empty()) std::memcpy(c->multi_host, table_.data(), table_.size());
        MD_TRY(dev_alloc(c, c->multi_dev, bytes));
        HIP_TRY(hipMemcpyAsync(c->multi_dev.p, c->multi_host, bytes, hipMemcpyHostToDevice, c->stream));
        for (auto &f : steps_) f(c->stream, static_cast<char *>(c->multi_dev.p));
        HIP_TRY(hipGetLastError());
        return MDLTS_OK;
    }
};

// every simulation's flags block to its pinned readback (the first `bytes`
// of it) after the next synchronisation: one collecting launch, one copy
mdlts_status collect_flags(mdlts_ctx *c, MultiPhase &ph, mdlts_sim *const *sims, const std::vector<int> &which)
{
    const size_t row = kFlagBytes;
    MD_TRY(dev_alloc(c, c->flags_dev, which.size() * row));
    const size_t bytes = which.size() * row;
    if (c->flags_host_bytes < bytes) {
        if (c->flags_host) (void)hipHostFree(c->flags_host);
        c->flags_host = nullptr;
        c->flags_host_bytes = 0;
        const size_t nb = std::max(bytes + bytes / 4, (size_t)16 << 10);
        if (hipHostMalloc(&c->flags_host, nb, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->flags_host = nullptr;
            return MDLTS_ENOMEM;
        }
        c->flags_host_bytes = nb;
    }
    for (size_t r = 0; r < which.size(); r++)
        ph.add(CopyFlagsOp{P<int>(sims[which[r]]->flags), P<int>(c->flags_dev) + r * (row / sizeof(int))}, 1);
    void *dst = c->flags_host, *src = c->flags_dev.p;
    ph.then([=](hipStream_t st, char *) { (void)hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st); });
    return MDLTS_OK;
}

void distribute_flags(mdlts_ctx *c, mdlts_sim *const *sims, const std::vector<int> &which, size_t bytes)
{
    for (size_t r = 0; r < which.size(); r++)
        std::memcpy(sims[which[r]]->pin, static_cast<char *>(c->flags_host) + r * kFlagBytes, bytes);
}

// ops of the kernel variants chosen at run time
template <typename T>
void add_indicator(MultiPhase &ph, const mdlts_sim *s, const IndArgs &a)
{
    const long long nb = nblocks((long long)s->E);
    const bool f = a.full != 0;
    switch (s->desc.dim * 10 + s->desc.order) {
    case 21: f ? ph.add(IndicatorOp<2, 1, T, true>{a}, nb) : ph.add(IndicatorOp<2, 1, T, false>{a}, nb); break;
    case 22: f ? ph.add(IndicatorOp<2, 2, T, true>{a}, nb) : ph.add(IndicatorOp<2, 2, T, false>{a}, nb); break;
    case 23: f ? ph.add(IndicatorOp<2, 3, T, true>{a}, nb) : ph.add(IndicatorOp<2, 3, T, false>{a}, nb); break;
    case 31: f ? ph.add(IndicatorOp<3, 1, T, true>{a}, nb) : ph.add(IndicatorOp<3, 1, T, false>{a}, nb); break;
    case 32: f ? ph.add(IndicatorOp<3, 2, T, true>{a}, nb) : ph.add(IndicatorOp<3, 2, T, false>{a}, nb); break;
    case 33: f ? ph.add(IndicatorOp<3, 3, T, true>{a}, nb) : ph.add(IndicatorOp<3, 3, T, false>{a}, nb); break;
    default: break;
    }
}

template <typename T>
void add_transfer(MultiPhase &ph, const mdlts_sim *s, const XferArgs &a)
{
    const long long nb = nblocks((long long)a.E_new);
    switch (s->desc.dim * 10 + s->desc.order) {
    case 21: ph.add(TransferOp<2, 1, T>{a}, nb); break;
    case 22: ph.add(TransferOp<2, 2, T>{a}, nb); break;
    case 23: ph.add(TransferOp<2, 3, T>{a}, nb); break;
    case 31: ph.add(TransferOp<3, 1, T>{a}, nb); break;
    case 32: ph.add(TransferOp<3, 2, T>{a}, nb); break;
    case 33: ph.add(TransferOp<3, 3, T>{a}, nb); break;
    default: break;
    }
}

// The two halves of mdlts_batch_adapt for two or more simulations: the same
// kernels with the same arguments as the per-simulation sequence, so the
// results are bitwise the same; what changes is that each step of all
// simulations is one launch per kernel variant (a few tens of launches per
// call instead of a few tens per simulation).
// First half: canonical state, indicator, marking, 2:1 closure, coarsening,
// counts and their scan; the counts arrive in each pin after the caller's
// synchronisation.
mdlts_status multi_adapt_count(mdlts_ctx *c, mdlts_sim *const *sims, int n, double tau_refine, double tau_coarsen)
{
    MultiPhase ph;
    // flags blocks cleared, grouped states gathered to canonical order
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        MD_TRY(dev_alloc(c, s->flags, kFlagBytes));
        ph.add(ClearFlagsOp{P<int>(s->flags)}, 1);
        if (s->state_grouped) {
            const int E = (int)s->E;
            MD_TRY(alloc_canonical_state(s));
            const long long stride = (long long)s->np * s->cap;
            const int parity = (int)(s->n_since_assign & 1);
            if (s->desc.precision == MDLTS_FP64)
                ph.add(GatherOp<double>{E, s->np, s->cap, stride, P<int>(s->perm), P<int>(s->cnt_ge_d), parity,
                                        P<double>(s->u_s), P<double>(s->v_s), P<double>(s->u_c), P<double>(s->v_c),
                                        nullptr},
                       nblocks(E));
            else
                ph.add(GatherOp<float>{E, s->np, s->cap, stride, P<int>(s->perm), P<int>(s->cnt_ge_d), parity,
                                       P<float>(s->u_s), P<float>(s->v_s), P<float>(s->u_c), P<float>(s->v_c),
                                       nullptr},
                       nblocks(E));
            s->state_grouped = false;
        }
    }
    ph.step();
    // indicator (as run_indicator)
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        MD_TRY(dev_alloc(c, s->eta_c, (size_t)E * sizeof(double)));
        IndArgs a;
        std::memset(&a, 0, sizeof(a));
        a.u = s->u_c.p;
        a.key = s->key_c.p;
        a.face = P<uint32_t>(s->face_c);
        a.fine = P<uint32_t>(s->fine_c);
        a.E = E;
        a.p = s->desc.order;
        for (int k = 0; k < 3; k++) { a.h0[k] = s->h0[k]; a.Dk[k] = s->Dk[k]; a.Dx[k] = s->Dx[k]; }
        a.full = s->dfull ? 1 : 0;
        fill_ref(s->ref, a.ref);
        a.eta = P<double>(s->eta_c);
        a.eta_max_bits = MD_FLAG(s, unsigned long long, eta_max_bits);
        a.nonfinite = MD_FLAG(s, int, eta_nonfinite);
        if (s->desc.precision == MDLTS_FP64) add_indicator<double>(ph, s, a);
        else add_indicator<float>(ph, s, a);
        s->eta_valid = true;
    }
    ph.step();
    // marking (as adapt_count)
    int passes = 0;
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const int nb4 = (E + 1023) / 1024;
        MD_TRY(dev_alloc(c, s->refine, (size_t)E));
        MD_TRY(dev_alloc(c, s->cflag, (size_t)E));
        MD_TRY(dev_alloc(c, s->cnt, (size_t)E * sizeof(int)));
        MD_TRY(dev_alloc(c, s->off, (size_t)E * sizeof(int)));
        MD_TRY(dev_alloc(c, s->bsums, (size_t)(nb4 + 1) * sizeof(int)));
        const MeshGeo g = geo_of(s);
        if (s->desc.dim == 2)
            ph.add(AmrMarkOp<2>{E, g, P<uint32_t>(s->key_c), P<double>(s->eta_c), tau_refine, P<uint8_t>(s->refine)},
                   nblocks(E));
        else
            ph.add(AmrMarkOp<3>{E, g, P<uint64_t>(s->key_c), P<double>(s->eta_c), tau_refine, P<uint8_t>(s->refine)},
                   nblocks(E));
        passes = std::max(passes, s->desc.max_depth);
    }
    ph.step();
    // 2:1 closure: max_depth passes per simulation
    for (int pass = 0; pass < passes; pass++) {
        for (int q = 0; q < n; q++) {
            mdlts_sim *s = sims[q];
            if (pass >= s->desc.max_depth) continue;
            const int E = (int)s->E;
            if (s->desc.dim == 2) ph.add(AmrCloseOp<2>{E, P<uint32_t>(s->face_c), P<uint8_t>(s->refine)}, nblocks(E));
            else ph.add(AmrCloseOp<3>{E, P<uint32_t>(s->face_c), P<uint8_t>(s->refine)}, nblocks(E));
        }
        ph.step();
    }
    // coarsening flags, then counts with their block scan, then the scan of
    // the block sums
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        if (s->desc.dim == 2)
            ph.add(AmrCoarsenOp<2>{E, P<uint32_t>(s->key_c), P<double>(s->eta_c), tau_coarsen, P<uint8_t>(s->refine),
                                   P<uint32_t>(s->face_c), P<uint8_t>(s->cflag)},
                   nblocks(E));
        else
            ph.add(AmrCoarsenOp<3>{E, P<uint64_t>(s->key_c), P<double>(s->eta_c), tau_coarsen, P<uint8_t>(s->refine),
                                   P<uint32_t>(s->face_c), P<uint8_t>(s->cflag)},
                   nblocks(E));
    }
    ph.step();
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const int nb4 = (E + 1023) / 1024;
        unsigned long long *tallies = MD_FLAG(s, unsigned long long, tallies);
        if (s->desc.dim == 2)
            ph.add(AmrCountScanOp<2>{E, P<uint32_t>(s->key_c), P<uint8_t>(s->refine), P<uint8_t>(s->cflag),
                                     P<int>(s->cnt), P<int>(s->off), P<int>(s->bsums), tallies},
                   nb4);
        else
            ph.add(AmrCountScanOp<3>{E, P<uint64_t>(s->key_c), P<uint8_t>(s->refine), P<uint8_t>(s->cflag),
                                     P<int>(s->cnt), P<int>(s->off), P<int>(s->bsums), tallies},
                   nb4);
    }
    ph.step();
    for (int q = 0; q < n; q++) {
        mdlts_sim *s = sims[q];
        const int nb4 = ((int)s->E + 1023) / 1024;
        ph.add(ScanSumsOp{nb4, P<int>(s->bsums), MD_FLAG(s, int, total)}, 1);
    }
    ph.step();
    std::vector<int> all(n);
    for (int q = 0; q < n; q++) all[q] = q;
    MD_TRY(collect_flags(c, ph, sims, all));
    return ph.run(c);
}

// Second half, for the simulations in `which` (their counts are on the
// host): new leaves, transfer, face tables, levels and grouping (as
// adapt_emit, device_faces and levels_enqueue); the flags with the level
// counts arrive in each pin after the caller's synchronisation.
mdlts_status multi_adapt_emit(mdlts_ctx *c, mdlts_sim *const *sims, const std::vector<int> &which,
                              const double *dt_barrier)
{
    MultiPhase ph;
    // new leaf keys and the transfer map
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const int E_new = s->pin->total;
        if (E_new <= 0 || E_new >= (1 << 27)) return MDLTS_EINVAL;
        if (s->desc.dim == 2) {
            MD_TRY(dev_alloc(c, s->key_n, (size_t)E_new * sizeof(uint32_t)));
        } else {
            MD_TRY(dev_alloc(c, s->key_n, (size_t)E_new * sizeof(uint64_t)));
        }
        MD_TRY(dev_alloc(c, s->xk, (size_t)E_new));
        MD_TRY(dev_alloc(c, s->xs, (size_t)E_new * sizeof(int32_t)));
        MD_TRY(dev_alloc(c, s->xc, (size_t)E_new));
        if (s->desc.dim == 2)
            ph.add(AmrEmitOp<2>{E, P<uint32_t>(s->key_c), P<uint8_t>(s->refine), P<uint8_t>(s->cflag), P<int>(s->cnt),
                                P<int>(s->off), P<int>(s->bsums), P<uint32_t>(s->key_n), P<uint8_t>(s->xk),
                                P<int32_t>(s->xs), P<uint8_t>(s->xc)},
                   nblocks(E));
        else
            ph.add(AmrEmitOp<3>{E, P<uint64_t>(s->key_c), P<uint8_t>(s->refine), P<uint8_t>(s->cflag), P<int>(s->cnt),
                                P<int>(s->off), P<int>(s->bsums), P<uint64_t>(s->key_n), P<uint8_t>(s->xk),
                                P<int32_t>(s->xs), P<uint8_t>(s->xc)},
                   nblocks(E));
    }
    ph.step();
    // transfer of u and v to the new leaves (as run_transfer)
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const int E_new = s->pin->total;
        const size_t bytes = (size_t)E_new * s->np * s->tsize;
        MD_TRY(dev_alloc(c, s->tmp_u, bytes));
        MD_TRY(dev_alloc(c, s->tmp_v, bytes));
        XferArgs a;
        std::memset(&a, 0, sizeof(a));
        a.u_old = s->u_c.p;
        a.v_old = s->v_c.p;
        a.u_new = s->tmp_u.p;
        a.v_new = s->tmp_v.p;
        a.E_old = E;
        a.E_new = E_new;
        a.kind = P<uint8_t>(s->xk);
        a.src = P<int32_t>(s->xs);
        a.child = P<uint8_t>(s->xc);
        fill_ref(s->ref, a.ref);
        if (s->desc.precision == MDLTS_FP64) add_transfer<double>(ph, s, a);
        else add_transfer<float>(ph, s, a);
        std::swap(s->u_c, s->tmp_u);
        std::swap(s->v_c, s->tmp_v);
        std::swap(s->key_c, s->key_n);
        s->E = (size_t)E_new;
        s->tree_rev++;
        s->host_forest_valid = false;
        s->levels_valid = false;
        s->eta_valid = false;
    }
    ph.step();
    // face tables of the new leaves (as device_faces)
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const int dim = s->desc.dim;
        const int n_roots = s->desc.n[0] * s->desc.n[1] * (dim == 3 ? s->desc.n[2] : 1);
        MD_TRY(dev_alloc(c, s->root_start, (size_t)(n_roots + 1) * sizeof(int)));
        MD_TRY(dev_alloc(c, s->mkey, (size_t)E * sizeof(uint32_t)));
        MD_TRY(dev_alloc(c, s->face_c, (size_t)2 * dim * E * sizeof(uint32_t)));
        MD_TRY(dev_alloc(c, s->fine_c, (size_t)2 * dim * E * n_sub(s) * sizeof(uint32_t)));
        const MeshGeo g = geo_of(s);
        if (dim == 2)
            ph.add(MeshIndexOp<2>{E, n_roots, g, P<uint32_t>(s->key_c), P<int>(s->root_start), P<uint32_t>(s->mkey)},
                   nblocks(E));
        else
            ph.add(MeshIndexOp<3>{E, n_roots, g, P<uint64_t>(s->key_c), P<int>(s->root_start), P<uint32_t>(s->mkey)},
                   nblocks(E));
    }
    ph.step();
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        const MeshGeo g = geo_of(s);
        int *bad = MD_FLAG(s, int, face_bad);
        if (s->desc.dim == 2)
            ph.add(MeshFacesOp<2>{E, g, P<uint32_t>(s->key_c), P<int>(s->root_start), P<uint32_t>(s->mkey),
                                  P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c), bad},
                   nblocks(2ll * 2 * E));
        else
            ph.add(MeshFacesOp<3>{E, g, P<uint64_t>(s->key_c), P<int>(s->root_start), P<uint32_t>(s->mkey),
                                  P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c), bad},
                   nblocks(2ll * 3 * E));
    }
    ph.step();
    // CFL levels (as levels_enqueue with the CFL criterion only)
    for (size_t r = 0; r < which.size(); r++) {
        mdlts_sim *s = sims[which[r]];
        const double dt = dt_barrier[which[r]];
        if ((uint64_t)2 * s->np * (((uint64_t)s->E + 63) / 64 * 64) * s->tsize > 0xffffffffull) return MDLTS_ENOMEM;
        s->version++;
        s->levels_valid = false;
        s->levels_plain_pending = true;
        const int E = (int)s->E;
        const int nb = nblocks(E);
        MD_TRY(dev_alloc(c, s->level_c, (size_t)E));
        MD_TRY(dev_alloc(c, s->cfl_c, (size_t)E * sizeof(double)));
        MD_TRY(dev_alloc(c, s->hist, (size_t)nb * kMaxLevels * sizeof(int)));
        MD_TRY(dev_alloc(c, s->cnt_ge_d, kMaxLevels * sizeof(int)));
        MD_TRY(dev_alloc(c, s->perm, (size_t)E * sizeof(int)));
        MD_TRY(dev_alloc(c, s->inv, (size_t)E * sizeof(int)));
        LevelArgs la;
        std::memset(&la, 0, sizeof(la));
        la.key = s->key_c.p;
        la.face = P<uint32_t>(s->face_c);
        la.E = E;
        la.dim = s->desc.dim;
        la.n_levels = s->desc.n_levels;
        la.force_level = -1;
        la.dt_bar = dt;
        for (int k = 0; k < 3; k++) { la.h0[k] = s->h0[k]; la.Dk[k] = s->Dk[k]; }
        std::memcpy(la.G, s->G, sizeof(la.G));
        if (s->dfull) {
            if (s->otab_dirty || !s->otab_d.p) {
                MD_TRY(dev_alloc(c, s->otab_d, s->otab.size() * sizeof(double)));
                HIP_TRY(hipMemcpyAsync(s->otab_d.p, s->otab.data(), s->otab.size() * sizeof(double),
                                       hipMemcpyHostToDevice, c->stream));
                s->otab_dirty = false;
            }
            la.otab = P<double>(s->otab_d);
        }
        la.level = P<uint8_t>(s->level_c);
        la.cfl = P<double>(s->cfl_c);
        la.hist = P<int>(s->hist);
        la.bad = MD_FLAG(s, int, level_bad);
        if (s->desc.dim == 2) ph.add(LevelsOp<2>{la}, nb);
        else ph.add(LevelsOp<3>{la}, nb);
    }
    ph.step();
    for (int q : which) {
        mdlts_sim *s = sims[q];
        ph.add(LevelScanOp{P<int>(s->hist), nblocks((long long)s->E), s->desc.n_levels, P<int>(s->cnt_ge_d),
                           MD_FLAG(s, int, cnt_ge)},
               1);
    }
    ph.step();
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        ph.add(LevelScatterOp{P<uint8_t>(s->level_c), E, P<int>(s->hist), P<int>(s->perm), P<int>(s->inv)},
               nblocks(E));
    }
    ph.step();
    // grouped tables and state (as the rest of levels_enqueue and to_grouped)
    for (int q : which) {
        mdlts_sim *s = sims[q];
        const int E = (int)s->E;
        s->cap = (E + 63) / 64 * 64;  // whole blocks of the grouped layout
        const size_t ksz = s->desc.dim == 2 ? 4 : 8;
        MD_TRY(dev_alloc(c, s->key_s, (size_t)s->cap * ksz));
        MD_TRY(dev_alloc(c, s->nbr_s, (size_t)s->cap * 2 * s->desc.dim * sizeof(uint32_t)));
        MD_TRY(dev_alloc(c, s->fine_s, (size_t)s->cap * 2 * s->desc.dim * n_sub(s) * sizeof(uint32_t)));
        if (s->desc.dim == 2)
            ph.add(RemapOp<uint32_t, 2>{E, 4, P<int>(s->perm), P<int>(s->inv), P<uint8_t>(s->level_c),
                                        P<uint32_t>(s->key_c), P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c),
                                        P<uint32_t>(s->key_s), P<uint32_t>(s->nbr_s), P<uint32_t>(s->fine_s), s->cap},
                   nblocks(E));
        else
            ph.add(RemapOp<uint64_t, 4>{E, 6, P<int>(s->perm), P<int>(s->inv), P<uint8_t>(s->level_c),
                                        P<uint64_t>(s->key_c), P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c),
                                        P<uint64_t>(s->key_s), P<uint32_t>(s->nbr_s), P<uint32_t>(s->fine_s), s->cap},
                   nblocks(E));
        const size_t sbytes = (size_t)s->cap * s->np * s->tsize;
        MD_TRY(dev_alloc(c, s->u_s, 2 * sbytes));
        MD_TRY(dev_alloc(c, s->v_s, sbytes));
        if (s->desc.precision == MDLTS_FP64)
            ph.add(PermuteOp<double>{E, s->np, s->cap, P<int>(s->perm), P<double>(s->u_c), P<double>(s->v_c),
                                     P<double>(s->u_s), P<double>(s->v_s)},
                   nblocks(E));
        else
            ph.add(PermuteOp<float>{E, s->np, s->cap, P<int>(s->perm), P<float>(s->u_c), P<float>(s->v_c),
                                    P<float>(s->u_s), P<float>(s->v_s)},
                   nblocks(E));
        s->state_grouped = true;
        s->n_since_assign = 0;
    }
    ph.step();
    MD_TRY(collect_flags(c, ph, sims, which));
    return ph.run(c);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *mdlts_strerror(mdlts_status s)
{
    switch (s) {
    case MDLTS_OK: return "ok";
    case MDLTS_EINVAL: return "invalid argument";
    case MDLTS_ENOMEM: return "device allocation failed";
    case MDLTS_EDEVICE: return "device error";
    case MDLTS_EUNSTABLE: return "more LTS levels needed than configured, or non-finite state";
    case MDLTS_ESTATE: return "call out of order";
    case MDLTS_EBUSY: return "simulation is busy";
    }
    return "unknown status";
}

mdlts_status mdlts_ctx_create(int device, void *hip_stream, const mdlts_allocator *alloc, mdlts_ctx **out)
{
    return abi_guard([&]() -> mdlts_status {
        if (!out) return MDLTS_EINVAL;
        *out = nullptr;
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MDLTS_EINVAL;
        if (alloc && (!alloc->alloc || !alloc->free)) return MDLTS_EINVAL;
        HIP_TRY(hipSetDevice(device));
        void *scr = nullptr;
        MD_TRY(scratch_address(device, &scr));
        mdlts_ctx *c = new (std::nothrow) mdlts_ctx;
        if (!c) return MDLTS_ENOMEM;
        c->device = device;
        c->scratch = scr;
        c->stream = static_cast<hipStream_t>(hip_stream);
        if (alloc) {
            c->alloc = *alloc;
            c->has_alloc = true;
        }
        *out = c;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_ctx_destroy(mdlts_ctx *ctx)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx) return MDLTS_EINVAL;
        if (ctx->n_sims > 0) return MDLTS_EBUSY;
        free_plan(ctx, ctx->batch);
        if (ctx->stage_done) (void)hipEventSynchronize(ctx->stage_done);
        if (ctx->stage) (void)hipHostFree(ctx->stage);
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->multi_host) (void)hipHostFree(ctx->multi_host);
        if (ctx->flags_host) (void)hipHostFree(ctx->flags_host);
        (void)dev_free(ctx, ctx->multi_dev);
        (void)dev_free(ctx, ctx->flags_dev);
        if (ctx->stage_done) (void)hipEventDestroy(ctx->stage_done);
        delete ctx;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_sync(mdlts_ctx *ctx)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx) return MDLTS_EINVAL;
        return sync(ctx);
    });
}

mdlts_status mdlts_sim_create(mdlts_ctx *ctx, const mdlts_mesh_desc *desc, mdlts_sim **out)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx || !out || !valid_desc(desc)) return MDLTS_EINVAL;
        *out = nullptr;
        mdlts_sim *s = new (std::nothrow) mdlts_sim;
        if (!s) return MDLTS_ENOMEM;
        s->ctx = ctx;
        ctx->n_sims++;
        if (hipHostMalloc(reinterpret_cast<void **>(&s->pin), sizeof(PinnedReadback), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->pin = nullptr;
            mdlts_sim_destroy(s);
            return MDLTS_ENOMEM;
        }
        std::memset(s->pin, 0, sizeof(PinnedReadback));
        s->desc = *desc;
        if (desc->dim == 2) { s->desc.n[2] = 1; s->desc.len[2] = 1.0; }
        s->np = 1;
        for (int k = 0; k < desc->dim; k++) s->np *= desc->order + 1;
        s->tsize = desc->precision == MDLTS_FP64 ? 8 : 4;
        for (int k = 0; k < 3; k++) s->h0[k] = s->desc.len[k] / (double)s->desc.n[k];
        make_ref_tables(desc->order, s->ref);
        // default penalty per degree (coercive: Q2 needs gamma > 2, Q3 > 5)
        s->gamma = desc->order == 1 ? 2.0 : desc->order == 2 ? 4.0 : 8.0;
        mdlts_status st = compute_G(s);
        Forest F;
        forest_from_desc(&s->desc, F);
        F.init_roots();
        if (st == MDLTS_OK && !F.build_faces()) st = MDLTS_EINVAL;
        if (st == MDLTS_OK) st = set_forest(s, std::move(F));
        if (st == MDLTS_OK) st = zero_canonical_state(s);
        if (st == MDLTS_OK) st = sync(ctx);
        if (st != MDLTS_OK) {
            mdlts_sim_destroy(s);
            return st;
        }
        *out = s;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_sim_destroy(mdlts_sim *s)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        (void)hipStreamSynchronize(c->stream);
        if (c->batch)
            for (mdlts_sim *m : c->batch->sims)
                if (m == s) {
                    free_plan(c, c->batch);
                    break;
                }
        free_plan(c, s->solo);
        DevBuf *bufs[] = {&s->key_c, &s->face_c, &s->fine_c, &s->u_c, &s->v_c, &s->level_c, &s->cfl_c, &s->eta_c,
                          &s->tmp_u, &s->tmp_v, &s->u_s, &s->v_s, &s->key_s, &s->nbr_s, &s->fine_s, &s->perm,
                          &s->inv, &s->hist, &s->cnt_ge_d, &s->flags, &s->xk, &s->xs, &s->xc, &s->stage,
                          &s->root_start, &s->mkey, &s->refine, &s->cflag, &s->cnt, &s->off, &s->bsums, &s->key_n,
                          &s->step_dev, &s->snap_u, &s->snap_v, &s->eta_t_c, &s->otab_d};
        mdlts_status st = MDLTS_OK;
        for (DevBuf *b : bufs)
            if (dev_free(c, *b) != MDLTS_OK) st = MDLTS_EDEVICE;
        for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
        if (s->pin) (void)hipHostFree(s->pin);
        c->n_sims--;
        delete s;
        return st;
    });
}

mdlts_status mdlts_set_tree(mdlts_sim *s, const uint8_t *bits, size_t n_bits)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || (!bits && n_bits)) return MDLTS_EINVAL;
        s->version++;
        Forest F;
        forest_from_desc(&s->desc, F);
        if (!F.parse_bits(bits, n_bits)) return MDLTS_EINVAL;
        if (F.size() >= (1u << 27)) return MDLTS_EINVAL;
        MD_TRY(set_forest(s, std::move(F)));
        return zero_canonical_state(s);
    });
}

mdlts_status mdlts_get_tree(mdlts_sim *s, uint8_t *bits, size_t cap, size_t *n_bits)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !n_bits) return MDLTS_EINVAL;
        MD_TRY(refresh_host_forest(s));
        std::vector<uint8_t> out;
        s->forest.write_bits(out);
        *n_bits = out.size();
        if (bits && cap >= out.size()) std::memcpy(bits, out.data(), out.size());
        return MDLTS_OK;
    });
}

mdlts_status mdlts_n_leaves(mdlts_sim *s, size_t *n)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !n) return MDLTS_EINVAL;
        *n = s->E;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_set_conductivity(mdlts_sim *s, const double D_sym[6], double gamma)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !(gamma > 0.0) || !std::isfinite(gamma)) return MDLTS_EINVAL;
        s->version++;
        Conductivity C;
        if (!parse_conductivity(D_sym, s->desc.dim, C)) return MDLTS_EINVAL;
        double G[4][4];
        if (!gershgorin_table(s->ref, gamma, G)) return MDLTS_EINVAL;
        std::vector<double> otab;
        if (C.full && !own_block_table(s->ref, s->desc.dim, s->h0, C, gamma, otab)) return MDLTS_EINVAL;
        for (int k = 0; k < 3; k++) {
            s->Dk[k] = k < s->desc.dim ? C.Dk[k] : 0.0;
            s->Dx[k] = C.Dx[k];
        }
        s->dfull = C.full;
        s->otab = std::move(otab);
        s->otab_dirty = C.full;
        s->gamma = gamma;
        s->step_dirty = true;
        std::memcpy(s->G, G, sizeof(G));
        s->levels_valid = s->levels_valid && false;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_set_ionic(mdlts_sim *s, const mdlts_ap_params *p)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !p) return MDLTS_EINVAL;
        s->version++;
        s->ap = *p;
        s->step_dirty = true;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_set_stimulus(mdlts_sim *s, const mdlts_stim_box *boxes, int n_boxes)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || n_boxes < 0 || n_boxes > kMaxStim || (n_boxes && !boxes)) return MDLTS_EINVAL;
        s->version++;
        s->stim.assign(boxes, boxes + n_boxes);
        s->step_dirty = true;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_set_state(mdlts_sim *s, const double *u, const double *v, size_t n_dof)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        s->version++;
        const size_t E = s->E;
        if (n_dof != E * (size_t)s->np) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        s->eta_valid = false;
        MD_TRY(to_canonical(s));
        MD_TRY(dev_alloc(c, s->stage, n_dof * sizeof(double)));
        const double *src[2] = {u, v};
        DevBuf *dst[2] = {&s->u_c, &s->v_c};
        for (int f = 0; f < 2; f++) {
            if (!src[f]) continue;
            HIP_TRY(hipMemcpyAsync(s->stage.p, src[f], n_dof * sizeof(double), hipMemcpyHostToDevice, c->stream));
            if (s->desc.precision == MDLTS_FP64)
                k_from_host<double><<<nblocks((long long)n_dof), kBlock, 0, c->stream>>>((int)E, s->np, P<double>(s->stage),
                                                                                        P<double>(*dst[f]));
            else
                k_from_host<float><<<nblocks((long long)n_dof), kBlock, 0, c->stream>>>((int)E, s->np, P<double>(s->stage),
                                                                                       P<float>(*dst[f]));
            HIP_TRY(hipGetLastError());
            MD_TRY(sync(c));  // the staging buffer is reused
        }
        if (s->levels_valid) MD_TRY(to_grouped(s));
        return sync(c);
    });
}

mdlts_status mdlts_get_state(mdlts_sim *s, double *u, double *v, size_t n_dof)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        const size_t E = s->E;
        if (n_dof != E * (size_t)s->np) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        const bool was_grouped = s->state_grouped;
        MD_TRY(to_canonical(s));
        MD_TRY(dev_alloc(c, s->stage, n_dof * sizeof(double)));
        double *dst[2] = {u, v};
        DevBuf *src[2] = {&s->u_c, &s->v_c};
        for (int f = 0; f < 2; f++) {
            if (!dst[f]) continue;
            if (s->desc.precision == MDLTS_FP64)
                k_to_host<double><<<nblocks((long long)n_dof), kBlock, 0, c->stream>>>((int)E, s->np, P<double>(*src[f]),
                                                                                      P<double>(s->stage));
            else
                k_to_host<float><<<nblocks((long long)n_dof), kBlock, 0, c->stream>>>((int)E, s->np, P<float>(*src[f]),
                                                                                     P<double>(s->stage));
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(dst[f], s->stage.p, n_dof * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            MD_TRY(sync(c));
        }
        // the grouped copy is still current: keep stepping from it
        if (was_grouped) s->state_grouped = true;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_set_time(mdlts_sim *s, double t)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !std::isfinite(t)) return MDLTS_EINVAL;
        s->version++;
        s->t_start = t;
        s->n_bar = 0;
        return MDLTS_OK;
    });
}

static mdlts_status assign_levels_impl(mdlts_sim *s, double dt_barrier, int force_level, int32_t *level_hist);

mdlts_status mdlts_assign_levels(mdlts_sim *s, double dt_barrier, int32_t *level_hist)
{
    return abi_guard([&]() -> mdlts_status {
        return assign_levels_impl(s, dt_barrier, -1, level_hist);
    });
}

mdlts_status mdlts_assign_uniform(mdlts_sim *s, double dt_barrier, int level, int32_t *level_hist)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || level < 0 || level >= s->desc.n_levels) return MDLTS_EINVAL;
        return assign_levels_impl(s, dt_barrier, level, level_hist);
    });
}

// Level assignment in two halves (so that several simulations can share the
// synchronisation): the CFL levels, grouping, grouped tables and the state
// permutation are enqueued; the level counts and the stability flag arrive
// in pin->cnt_ge / pin->level_bad after the next synchronisation.
static mdlts_status levels_enqueue(mdlts_sim *s, double dt_barrier, int force_level, const double *eta_t = nullptr,
                                   double tau_cell = 0.0, int b_cell = 0, bool own_flags = true)
{
    if (!(dt_barrier > 0.0) || !std::isfinite(dt_barrier)) return MDLTS_EINVAL;
    // the substep kernels address both u slots with 32-bit byte offsets
    if ((uint64_t)2 * s->np * (((uint64_t)s->E + 63) / 64 * 64) * s->tsize > 0xffffffffull) return MDLTS_ENOMEM;
    s->version++;
    s->levels_valid = false;
    s->levels_plain_pending = force_level < 0 && !eta_t;
    mdlts_ctx *c = s->ctx;
    const int E = (int)s->E;
    const int L = s->desc.n_levels;
    const int nb = nblocks(E);
    MD_TRY(to_canonical(s));
    MD_TRY(dev_alloc(c, s->level_c, (size_t)E));
    MD_TRY(dev_alloc(c, s->cfl_c, (size_t)E * sizeof(double)));
    MD_TRY(dev_alloc(c, s->hist, (size_t)nb * kMaxLevels * sizeof(int)));
    MD_TRY(dev_alloc(c, s->cnt_ge_d, kMaxLevels * sizeof(int)));
    MD_TRY(dev_alloc(c, s->perm, (size_t)E * sizeof(int)));
    MD_TRY(dev_alloc(c, s->inv, (size_t)E * sizeof(int)));
    if (own_flags) MD_TRY(flags_clear(s));
    LevelArgs la;
    std::memset(&la, 0, sizeof(la));
    la.key = s->key_c.p;
    la.face = P<uint32_t>(s->face_c);
    la.E = E;
    la.dim = s->desc.dim;
    la.n_levels = L;
    la.force_level = force_level;
    la.dt_bar = dt_barrier;
    la.eta_t = eta_t;
    la.tau_cell = tau_cell;
    la.b_cell = b_cell;
    for (int k = 0; k < 3; k++) { la.h0[k] = s->h0[k]; la.Dk[k] = s->Dk[k]; }
    std::memcpy(la.G, s->G, sizeof(la.G));
    if (s->dfull) {
        if (s->otab_dirty || !s->otab_d.p) {
            MD_TRY(dev_alloc(c, s->otab_d, s->otab.size() * sizeof(double)));
            HIP_TRY(hipMemcpyAsync(s->otab_d.p, s->otab.data(), s->otab.size() * sizeof(double), hipMemcpyHostToDevice,
                                   c->stream));
            s->otab_dirty = false;
        }
        la.otab = P<double>(s->otab_d);
    }
    la.level = P<uint8_t>(s->level_c);
    la.cfl = P<double>(s->cfl_c);
    la.hist = P<int>(s->hist);
    la.bad = MD_FLAG(s, int, level_bad);
    if (s->desc.dim == 2) k_levels<2><<<nb, kBlock, 0, c->stream>>>(la);
    else k_levels<3><<<nb, kBlock, 0, c->stream>>>(la);
    HIP_TRY(hipGetLastError());
    if (own_flags) HIP_TRY(hipMemcpyAsync(&s->pin->level_bad, la.bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    // (levels above the cap are clamped by k_levels, so what follows stays
    // well defined; the flag makes the assignment invalid afterwards)
    // the counts also go to the flags block, read back with the flags when
    // the caller collects them
    k_level_scan<<<1, kBlock, 0, c->stream>>>(P<int>(s->hist), nb, L, P<int>(s->cnt_ge_d), MD_FLAG(s, int, cnt_ge));
    k_level_scatter<<<nb, kBlock, 0, c->stream>>>(P<uint8_t>(s->level_c), E, P<int>(s->hist), P<int>(s->perm),
                                                   P<int>(s->inv));
    // grouped tables
    s->cap = (E + 63) / 64 * 64;  // whole blocks of the grouped layout
    const size_t ksz = s->desc.dim == 2 ? 4 : 8;
    MD_TRY(dev_alloc(c, s->key_s, (size_t)s->cap * ksz));
    MD_TRY(dev_alloc(c, s->nbr_s, (size_t)s->cap * 2 * s->desc.dim * sizeof(uint32_t)));
    MD_TRY(dev_alloc(c, s->fine_s, (size_t)s->cap * 2 * s->desc.dim * n_sub(s) * sizeof(uint32_t)));
    if (s->desc.dim == 2)
        k_remap<uint32_t, 2><<<nb, kBlock, 0, c->stream>>>(E, 4, P<int>(s->perm), P<int>(s->inv),
                                                            P<uint8_t>(s->level_c), P<uint32_t>(s->key_c),
                                                            P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c),
                                                            P<uint32_t>(s->key_s), P<uint32_t>(s->nbr_s),
                                                            P<uint32_t>(s->fine_s), s->cap);
    else
        k_remap<uint64_t, 4><<<nb, kBlock, 0, c->stream>>>(E, 6, P<int>(s->perm), P<int>(s->inv),
                                                            P<uint8_t>(s->level_c), P<uint64_t>(s->key_c),
                                                            P<uint32_t>(s->face_c), P<uint32_t>(s->fine_c),
                                                            P<uint64_t>(s->key_s), P<uint32_t>(s->nbr_s),
                                                            P<uint32_t>(s->fine_s), s->cap);
    const size_t sbytes = (size_t)s->cap * s->np * s->tsize;
    MD_TRY(dev_alloc(c, s->u_s, 2 * sbytes));
    MD_TRY(dev_alloc(c, s->v_s, sbytes));
    HIP_TRY(hipGetLastError());
    if (own_flags)
        HIP_TRY(hipMemcpyAsync(s->pin->cnt_ge, s->cnt_ge_d.p, kMaxLevels * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    return to_grouped(s);
}

// after the synchronisation: level counts on the host, time base, validity
static mdlts_status levels_finish(mdlts_sim *s, double dt_barrier, int32_t *level_hist)
{
    if (s->pin->level_bad) return MDLTS_EUNSTABLE;
    const int L = s->desc.n_levels;
    s->cnt_ge.assign(s->pin->cnt_ge, s->pin->cnt_ge + L);
    s->lmax = 0;
    for (int l = 0; l < L; l++)
        if (s->cnt_ge[l] > 0) s->lmax = l;
    if (level_hist)
        for (int l = 0; l < L; l++) level_hist[l] = s->cnt_ge[l] - (l + 1 < L ? s->cnt_ge[l + 1] : 0);
    if (dt_barrier != s->dt_bar) {
        s->t_start = s->t_start + (double)s->n_bar * s->dt_bar;
        s->n_bar = 0;
        s->dt_bar = dt_barrier;
    }
    s->levels_valid = true;
    s->levels_plain = s->levels_plain_pending;
    s->step_dirty = true;
    return MDLTS_OK;
}

static mdlts_status assign_levels_impl(mdlts_sim *s, double dt_barrier, int force_level, int32_t *level_hist)
{
    if (!s) return MDLTS_EINVAL;
    MD_TRY(levels_enqueue(s, dt_barrier, force_level));
    MD_TRY(sync(s->ctx));
    return levels_finish(s, dt_barrier, level_hist);
}

mdlts_status mdlts_assign_levels_auto(mdlts_sim *s, double *dt_barrier, int32_t *level_hist)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !dt_barrier) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        const int E = (int)s->E;
        // CFL of every leaf (the level pass with every leaf forced to level 0),
        // then its minimum
        MD_TRY(levels_enqueue(s, 1.0, 0));
        unsigned long long *mb = MD_FLAG(s, unsigned long long, eta_max_bits);
        const unsigned long long init = 0x7fefffffffffffffull;  // largest finite double
        HIP_TRY(hipMemcpyAsync(mb, &init, 8, hipMemcpyHostToDevice, c->stream));
        k_min_positive<<<nblocks(E), kBlock, 0, c->stream>>>(E, P<double>(s->cfl_c), mb);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&s->pin->eta_max_bits, mb, 8, hipMemcpyDeviceToHost, c->stream));
        MD_TRY(sync(c));
        double cfl_min;
        std::memcpy(&cfl_min, &s->pin->eta_max_bits, 8);
        if (!(cfl_min > 0.0) || !std::isfinite(cfl_min)) return MDLTS_EUNSTABLE;
        // every leaf within the configured levels, off the power-of-two ties
        const double dt = std::ldexp(cfl_min, s->desc.n_levels - 1) * (1.0 - std::ldexp(1.0, -20));
        *dt_barrier = dt;
        return assign_levels_impl(s, dt, -1, level_hist);
    });
}

mdlts_status mdlts_rvt_snapshot(mdlts_sim *s)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        const bool was_grouped = s->state_grouped;
        MD_TRY(to_canonical(s));
        const size_t bytes = s->E * s->np * s->tsize;
        MD_TRY(dev_alloc(c, s->snap_u, bytes));
        MD_TRY(dev_alloc(c, s->snap_v, bytes));
        HIP_TRY(hipMemcpyAsync(s->snap_u.p, s->u_c.p, bytes, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(s->snap_v.p, s->v_c.p, bytes, hipMemcpyDeviceToDevice, c->stream));
        if (was_grouped) s->state_grouped = true;  // the grouped copy is untouched
        s->snap_t = s->t_start + (double)s->n_bar * s->dt_bar;
        s->snap_rev = s->tree_rev;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_rvt_indicator(mdlts_sim *s, double *eta_t, size_t n_leaves, double *eta_t_max)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        const size_t E = s->E;
        if (eta_t && n_leaves != E) return MDLTS_EINVAL;
        const double t_b = s->t_start + (double)s->n_bar * s->dt_bar;
        if (s->snap_rev != s->tree_rev || !(t_b > s->snap_t)) return MDLTS_ESTATE;
        mdlts_ctx *c = s->ctx;
        const bool was_grouped = s->state_grouped;
        MD_TRY(to_canonical(s));
        MD_TRY(dev_alloc(c, s->eta_t_c, E * sizeof(double)));
        MD_TRY(flags_clear(s));
        RvtArgs a;
        std::memset(&a, 0, sizeof(a));
        a.u_a = s->snap_u.p;
        a.v_a = s->snap_v.p;
        a.u_b = s->u_c.p;
        a.v_b = s->v_c.p;
        a.key = s->key_c.p;
        a.E = (int)E;
        for (int k = 0; k < 3; k++) a.h0[k] = s->h0[k];
        a.apk = s->ap.k; a.apa = s->ap.a; a.eps0 = s->ap.eps0; a.mu1 = s->ap.mu1; a.mu2 = s->ap.mu2;
        a.t_a = s->snap_t;
        a.t_b = t_b;
        a.n_stim = (int)s->stim.size();
        for (int b = 0; b < a.n_stim; b++) {
            const mdlts_stim_box &B = s->stim[b];
            for (int k = 0; k < 3; k++) { a.stim[b][k] = B.lo[k]; a.stim[b][3 + k] = B.hi[k]; }
            a.stim[b][6] = B.t_on; a.stim[b][7] = B.t_off; a.stim[b][8] = B.amp;
        }
        a.eta = P<double>(s->eta_t_c);
        a.eta_max_bits = MD_FLAG(s, unsigned long long, eta_max_bits);
        const int nb = nblocks((int)E);
        hipStream_t st = c->stream;
        switch (s->desc.dim * 100 + s->desc.order * 10 + (s->desc.precision == MDLTS_FP32 ? 1 : 0)) {
        case 210: k_rvt<2, 1, double><<<nb, kBlock, 0, st>>>(a); break;
        case 220: k_rvt<2, 2, double><<<nb, kBlock, 0, st>>>(a); break;
        case 310: k_rvt<3, 1, double><<<nb, kBlock, 0, st>>>(a); break;
        case 320: k_rvt<3, 2, double><<<nb, kBlock, 0, st>>>(a); break;
        case 211: k_rvt<2, 1, float><<<nb, kBlock, 0, st>>>(a); break;
        case 221: k_rvt<2, 2, float><<<nb, kBlock, 0, st>>>(a); break;
        case 311: k_rvt<3, 1, float><<<nb, kBlock, 0, st>>>(a); break;
        case 321: k_rvt<3, 2, float><<<nb, kBlock, 0, st>>>(a); break;
        case 230: k_rvt<2, 3, double><<<nb, kBlock, 0, st>>>(a); break;
        case 330: k_rvt<3, 3, double><<<nb, kBlock, 0, st>>>(a); break;
        case 231: k_rvt<2, 3, float><<<nb, kBlock, 0, st>>>(a); break;
        case 331: k_rvt<3, 3, float><<<nb, kBlock, 0, st>>>(a); break;
        default: return MDLTS_EINVAL;
        }
        HIP_TRY(hipGetLastError());
        if (eta_t) HIP_TRY(hipMemcpyAsync(eta_t, s->eta_t_c.p, E * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&s->pin->eta_max_bits, a.eta_max_bits, 8, hipMemcpyDeviceToHost, st));
        MD_TRY(sync(c));
        if (was_grouped) s->state_grouped = true;
        if (eta_t_max) std::memcpy(eta_t_max, &s->pin->eta_max_bits, 8);
        s->eta_t_rev = s->tree_rev;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_assign_levels_cell(mdlts_sim *s, double dt_barrier, double tau_cell, double dt_cell,
                                      int32_t *level_hist)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !(dt_cell > 0.0) || !std::isfinite(dt_cell) || !(dt_barrier > 0.0)) return MDLTS_EINVAL;
        if (s->eta_t_rev != s->tree_rev) return MDLTS_ESTATE;
        int b_cell = 0;  // ceil(log2(dt_barrier / dt_cell)) by exact scaling
        while (b_cell < 64 && std::ldexp(dt_barrier, -b_cell) > dt_cell) b_cell++;
        MD_TRY(levels_enqueue(s, dt_barrier, -1, P<double>(s->eta_t_c), tau_cell, b_cell));
        MD_TRY(sync(s->ctx));
        return levels_finish(s, dt_barrier, level_hist);
    });
}

mdlts_status mdlts_get_levels(mdlts_sim *s, int8_t *level, int32_t *perm, int32_t *cnt_ge, size_t n_leaves)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        if (!s->levels_valid) return MDLTS_ESTATE;
        if (n_leaves != s->E) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        if (level) HIP_TRY(hipMemcpyAsync(level, s->level_c.p, n_leaves, hipMemcpyDeviceToHost, c->stream));
        if (perm) HIP_TRY(hipMemcpyAsync(perm, s->perm.p, n_leaves * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        if (cnt_ge)
            for (size_t l = 0; l < s->cnt_ge.size(); l++) cnt_ge[l] = s->cnt_ge[l];
        return sync(c);
    });
}

mdlts_status mdlts_get_cfl(mdlts_sim *s, double *cfl, size_t n_leaves)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || !cfl) return MDLTS_EINVAL;
        if (!s->levels_valid) return MDLTS_ESTATE;
        if (n_leaves != s->E) return MDLTS_EINVAL;
        HIP_TRY(hipMemcpyAsync(cfl, s->cfl_c.p, n_leaves * sizeof(double), hipMemcpyDeviceToHost, s->ctx->stream));
        return sync(s->ctx);
    });
}

mdlts_status mdlts_step(mdlts_sim *s, int n_barriers)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s || n_barriers < 0) return MDLTS_EINVAL;
        if (!s->levels_valid || !s->state_grouped) return MDLTS_ESTATE;
        s->eta_valid = false;
        mdlts_ctx *c = s->ctx;
        if (!c->use_graphs) {
            if (s->desc.precision == MDLTS_FP64) return run_barriers<double>(s, n_barriers);
            return run_barriers<float>(s, n_barriers);
        }
        // a one-simulation plan of tile launches (one kernel variant: launched
        // directly, see run_batch_barriers)
        bool fresh = false;
        MD_TRY(prepare_plan(c, s->solo, &s, 1, &fresh));
        BatchPlan &P = *s->solo;
        if (P.prof != s->prof) {
            MD_TRY(drain_batch_events(P));
            P.prof = s->prof;
        }
        int remaining = n_barriers;
        if (!P.tuned) MD_TRY(autotune(c, P, &remaining));
        return run_batch_barriers(c, P, remaining);
    });
}

// the indicator on the device (canonical state, FP64 eta in eta_c); its
// maximum and non-finite flag arrive in pin after the next synchronisation
static mdlts_status indicator_enqueue(mdlts_sim *s, bool own_flags = true)
{
    mdlts_ctx *c = s->ctx;
    const size_t E = s->E;
    const bool was_grouped = s->state_grouped;
    MD_TRY(to_canonical(s));
    MD_TRY(dev_alloc(c, s->eta_c, E * sizeof(double)));
    if (own_flags) MD_TRY(flags_clear(s));
    unsigned long long *maxb = MD_FLAG(s, unsigned long long, eta_max_bits);
    int *nonf = MD_FLAG(s, int, eta_nonfinite);
    if (s->desc.precision == MDLTS_FP64) MD_TRY(run_indicator<double>(s, s->u_c.p, P<double>(s->eta_c), maxb, nonf));
    else MD_TRY(run_indicator<float>(s, s->u_c.p, P<double>(s->eta_c), maxb, nonf));
    // the non-finite flag and the maximum are adjacent: one copy
    static_assert(offsetof(PinnedReadback, eta_max_bits) == offsetof(PinnedReadback, eta_nonfinite) + sizeof(int),
                  "readback layout");
    if (own_flags)
        HIP_TRY(hipMemcpyAsync(&s->pin->eta_nonfinite, nonf, sizeof(int) + sizeof(unsigned long long),
                               hipMemcpyDeviceToHost, c->stream));
    // the grouped copy of the state is untouched
    if (was_grouped) s->state_grouped = true;
    s->eta_valid = true;
    return MDLTS_OK;
}

mdlts_status mdlts_indicator(mdlts_sim *s, double *eta, size_t n_leaves, double *eta_max)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        const size_t E = s->E;
        if (eta && n_leaves != E) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        MD_TRY(indicator_enqueue(s));
        if (eta) HIP_TRY(hipMemcpyAsync(eta, s->eta_c.p, E * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        MD_TRY(sync(c));
        if (eta_max) std::memcpy(eta_max, &s->pin->eta_max_bits, 8);
        return s->pin->eta_nonfinite ? MDLTS_EUNSTABLE : MDLTS_OK;
    });
}

mdlts_status mdlts_indicator_noalloc(mdlts_sim *s, double *eta, size_t n_leaves, double *eta_max)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        const size_t E = s->E;
        if (eta && n_leaves != E) return MDLTS_EINVAL;
        mdlts_ctx *c = s->ctx;
        if (!c->scratch) return MDLTS_EDEVICE;
        // scratch layout: [flags 256 B | eta E doubles | canonical u, if the
        // state is grouped], each part 256-byte aligned
        const auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
        const size_t eta_off = 256;
        const size_t u_off = eta_off + up(E * sizeof(double));
        const size_t need = u_off + (s->state_grouped ? up(E * (size_t)s->np * s->tsize) : 0);
        if (need > kScratchBytes) return MDLTS_ENOMEM;
        char *base = static_cast<char *>(c->scratch);
        unsigned long long *maxb = reinterpret_cast<unsigned long long *>(base);
        int *nonf = reinterpret_cast<int *>(base + 8);
        double *eta_d = reinterpret_cast<double *>(base + eta_off);
        hipStream_t st = c->stream;
        // the maximum (as bits of a non-negative double) and the flag start at 0
        k_clear_u32<<<1, 64, 0, st>>>(reinterpret_cast<uint32_t *>(base), 4);
        HIP_TRY(hipGetLastError());
        const void *u = s->u_c.p;
        if (s->state_grouped) {
            // the current slot in canonical order; the grouped state stays as is
            const int Ei = (int)E;
            const long long stride = (long long)s->np * s->cap;
            const int parity = (int)(s->n_since_assign & 1);
            void *uc = base + u_off;
            if (s->desc.precision == MDLTS_FP64)
                k_gather<double><<<nblocks(Ei), kBlock, 0, st>>>(Ei, s->np, s->cap, stride, P<int>(s->perm),
                                                                  P<int>(s->cnt_ge_d), parity, P<double>(s->u_s),
                                                                  nullptr, static_cast<double *>(uc), nullptr, nullptr);
            else
                k_gather<float><<<nblocks(Ei), kBlock, 0, st>>>(Ei, s->np, s->cap, stride, P<int>(s->perm),
                                                                 P<int>(s->cnt_ge_d), parity, P<float>(s->u_s),
                                                                 nullptr, static_cast<float *>(uc), nullptr, nullptr);
            HIP_TRY(hipGetLastError());
            u = uc;
        }
        if (s->desc.precision == MDLTS_FP64) MD_TRY(run_indicator<double>(s, u, eta_d, maxb, nonf));
        else MD_TRY(run_indicator<float>(s, u, eta_d, maxb, nonf));
        if (eta) HIP_TRY(hipMemcpyAsync(eta, eta_d, E * sizeof(double), hipMemcpyDeviceToHost, st));
        // the flag and the maximum into the simulation's pinned readback block
        HIP_TRY(hipMemcpyAsync(&s->pin->eta_nonfinite, nonf, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(&s->pin->eta_max_bits, maxb, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        MD_TRY(sync(c));
        if (eta_max) std::memcpy(eta_max, &s->pin->eta_max_bits, 8);
        return s->pin->eta_nonfinite ? MDLTS_EUNSTABLE : MDLTS_OK;
    });
}

mdlts_status mdlts_adapt(mdlts_sim *s, const double *eta, size_t n_leaves, double tau_refine, double tau_coarsen,
                         int64_t *n_refined, int64_t *n_coarsened)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        const size_t E = s->E;
        if (eta && n_leaves != E) return MDLTS_EINVAL;
        if (!eta && !s->eta_valid) return MDLTS_ESTATE;
        s->version++;
        mdlts_ctx *c = s->ctx;
        if (eta) {
            MD_TRY(copy_h2d(c, s->eta_c, eta, E));
            MD_TRY(sync(c));
        }
        MD_TRY(to_canonical(s));
        if (s->desc.dim == 2) MD_TRY(adapt_count<2>(s, tau_refine, tau_coarsen));
        else MD_TRY(adapt_count<3>(s, tau_refine, tau_coarsen));
        MD_TRY(sync(c));
        if (n_refined) *n_refined = (int64_t)s->pin->tallies[0];
        if (n_coarsened) *n_coarsened = (int64_t)s->pin->tallies[1];
        if (s->desc.dim == 2) MD_TRY(adapt_emit<2>(s));
        else MD_TRY(adapt_emit<3>(s));
        MD_TRY(sync(c));
        return s->pin->face_bad ? MDLTS_EINVAL : MDLTS_OK;
    });
}

mdlts_status mdlts_counters(mdlts_sim *s, uint64_t *dof_updates, double *t_sim)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        if (dof_updates) *dof_updates = s->dof_updates;
        if (t_sim) *t_sim = s->t_start + (double)s->n_bar * s->dt_bar;
        return MDLTS_OK;
    });
}

// event times of the step plan's launches, added to the simulation's
static mdlts_status drain_solo(mdlts_sim *s)
{
    if (!s->solo) return MDLTS_OK;
    BatchPlan &P = *s->solo;
    MD_TRY(drain_batch_events(P));
    s->prof_ms += P.prof_ms;
    s->prof_launches += P.prof_launches;
    s->prof_dof += P.prof_dof;
    P.prof_ms = 0.0;
    P.prof_launches = P.prof_dof = 0;
    return MDLTS_OK;
}

mdlts_status mdlts_profile(mdlts_sim *s, int enable)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        MD_TRY(drain_events(s));
        MD_TRY(drain_solo(s));
        s->prof = enable != 0;
        s->prof_ms = 0.0;
        s->prof_launches = s->prof_dof = 0;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_profile_read(mdlts_sim *s, double *substep_ms, uint64_t *n_launches, uint64_t *dof_updates)
{
    return abi_guard([&]() -> mdlts_status {
        if (!s) return MDLTS_EINVAL;
        MD_TRY(drain_events(s));
        MD_TRY(drain_solo(s));
        if (substep_ms) *substep_ms = s->prof_ms;
        if (n_launches) *n_launches = s->prof_launches;
        if (dof_updates) *dof_updates = s->prof_dof;
        s->prof_ms = 0.0;
        s->prof_launches = s->prof_dof = 0;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_batch_step(mdlts_ctx *ctx, mdlts_sim *const *sims, int n_sims, int n_barriers)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx || !sims || n_sims < 1 || n_barriers < 0) return MDLTS_EINVAL;
        for (int q = 0; q < n_sims; q++) {
            if (!sims[q] || sims[q]->ctx != ctx) return MDLTS_EINVAL;
            for (int r = 0; r < q; r++)
                if (sims[r] == sims[q]) return MDLTS_EINVAL;
            if (!sims[q]->levels_valid || !sims[q]->state_grouped) return MDLTS_ESTATE;
        }
        bool fresh = false;
        MD_TRY(prepare_plan(ctx, ctx->batch, sims, n_sims, &fresh));
        BatchPlan &P = *ctx->batch;
        int remaining = n_barriers;
        if (!P.tuned) MD_TRY(autotune(ctx, P, &remaining));
        MD_TRY(run_batch_barriers(ctx, P, remaining));
        return MDLTS_OK;
    });
}

mdlts_status mdlts_batch_adapt(mdlts_ctx *ctx, mdlts_sim *const *sims, int n_sims, double tau_refine,
                               double tau_coarsen, const double *dt_barrier)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx || !sims || n_sims < 1 || !dt_barrier) return MDLTS_EINVAL;
        for (int q = 0; q < n_sims; q++) {
            if (!sims[q] || sims[q]->ctx != ctx) return MDLTS_EINVAL;
            for (int r = 0; r < q; r++)
                if (sims[r] == sims[q]) return MDLTS_EINVAL;
            if (!(dt_barrier[q] > 0.0) || !std::isfinite(dt_barrier[q])) return MDLTS_EINVAL;
        }
        // A simulation whose leaves do not change keeps its levels when they are
        // the CFL levels of the same barrier step: no transfer, faces, levels or
        // regrouping; its grouped state (which the indicator only reads from a
        // canonical copy) stays in place, and its step plans stay valid.  The
        // results are bitwise those of the full sequence.
        std::vector<char> keep(n_sims);
        for (int q = 0; q < n_sims; q++)
            keep[q] = sims[q]->levels_valid && sims[q]->state_grouped && sims[q]->levels_plain &&
                      dt_barrier[q] == sims[q]->dt_bar;
        if (n_sims > 1) {
            // every step of all simulations in one launch per kernel variant
            MD_TRY(multi_adapt_count(ctx, sims, n_sims, tau_refine, tau_coarsen));
            MD_TRY(sync(ctx));
            std::vector<int> all(n_sims), change;
            for (int q = 0; q < n_sims; q++) all[q] = q;
            distribute_flags(ctx, sims, all, kFlagHead);
            for (int q = 0; q < n_sims; q++) {
                mdlts_sim *s = sims[q];
                keep[q] = keep[q] && s->pin->tallies[0] == 0 && s->pin->tallies[1] == 0 && s->pin->total == (int)s->E;
                if (keep[q]) s->state_grouped = true;
                else change.push_back(q);
            }
            if (!change.empty()) {
                for (int q : change) sims[q]->version++;
                MD_TRY(multi_adapt_emit(ctx, sims, change, dt_barrier));
                MD_TRY(sync(ctx));
                distribute_flags(ctx, sims, change, sizeof(PinnedReadback));
            }
        } else {
            // one simulation: its own launches (no tables to send)
            mdlts_sim *s = sims[0];
            // the adaptation works on the canonical copy of the state; the
            // gather that makes it current also clears the flags block (the
            // grouped copy stays valid if the leaves do not change)
            if (s->state_grouped) {
                MD_TRY(dev_alloc(ctx, s->flags, kFlagBytes));
                MD_TRY(to_canonical(s, flag_at<int>(s, 0)));
            } else {
                MD_TRY(flags_clear(s));
            }
            MD_TRY(indicator_enqueue(s, false));
            if (s->desc.dim == 2) MD_TRY(adapt_count<2>(s, tau_refine, tau_coarsen, false));
            else MD_TRY(adapt_count<3>(s, tau_refine, tau_coarsen, false));
            MD_TRY(flags_readback(s));
            MD_TRY(sync(ctx));
            keep[0] = keep[0] && s->pin->tallies[0] == 0 && s->pin->tallies[1] == 0 && s->pin->total == (int)s->E;
            if (keep[0]) {
                s->state_grouped = true;
            } else {
                s->version++;
                if (s->desc.dim == 2) MD_TRY(adapt_emit<2>(s, false));
                else MD_TRY(adapt_emit<3>(s, false));
                MD_TRY(levels_enqueue(s, dt_barrier[0], -1, nullptr, 0.0, 0, false));
                MD_TRY(flags_readback(s, true));
                MD_TRY(sync(ctx));
            }
        }
        mdlts_status first = MDLTS_OK;
        for (int q = 0; q < n_sims; q++) {
            mdlts_sim *s = sims[q];
            if (keep[q]) {
                if (first == MDLTS_OK && s->pin->eta_nonfinite) first = MDLTS_EUNSTABLE;
                continue;
            }
            mdlts_status st = s->pin->face_bad ? MDLTS_EINVAL : levels_finish(s, dt_barrier[q], nullptr);
            if (st == MDLTS_OK && s->pin->eta_nonfinite) st = MDLTS_EUNSTABLE;
            if (first == MDLTS_OK) first = st;
        }
        return first;
    });
}

mdlts_status mdlts_set_graphs(mdlts_ctx *ctx, int enable)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx) return MDLTS_EINVAL;
        ctx->use_graphs = enable != 0;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_batch_profile(mdlts_ctx *ctx, int enable)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx || !ctx->batch) return MDLTS_ESTATE;
        BatchPlan &P = *ctx->batch;
        MD_TRY(drain_batch_events(P));
        P.prof = enable != 0;
        P.prof_ms = 0.0;
        P.prof_launches = P.prof_dof = 0;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_batch_profile_read(mdlts_ctx *ctx, double *substep_ms, uint64_t *n_launches,
                                      uint64_t *dof_updates, int *block, int *per_cu)
{
    return abi_guard([&]() -> mdlts_status {
        if (!ctx || !ctx->batch) return MDLTS_ESTATE;
        BatchPlan &P = *ctx->batch;
        MD_TRY(drain_batch_events(P));
        if (substep_ms) *substep_ms = P.prof_ms;
        if (n_launches) *n_launches = P.prof_launches;
        if (dof_updates) *dof_updates = P.prof_dof;
        if (block) *block = P.block;
        if (per_cu) *per_cu = P.per_cu;
        P.prof_ms = 0.0;
        P.prof_launches = P.prof_dof = 0;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_cfl_bound(const mdlts_mesh_desc *desc, const double D_sym[6], double gamma, int depth,
                             double *cfl_min)
{
    return abi_guard([&]() -> mdlts_status {
        if (!valid_desc(desc) || !cfl_min || depth < 0 || depth > desc->max_depth || !(gamma > 0.0)) return MDLTS_EINVAL;
        Conductivity C;
        if (!parse_conductivity(D_sym, desc->dim, C)) return MDLTS_EINVAL;
        RefTables R;
        make_ref_tables(desc->order, R);
        double G[4][4];
        if (!gershgorin_table(R, gamma, G)) return MDLTS_EINVAL;
        // Face kinds a leaf of this depth can have in direction k: no finer
        // neighbour at the depth cap, no coarser one at depth 0, both faces on
        // the boundary only for a single root across the box, and below the
        // roots one face always sees the sibling cell (same size or finer).
        double s = 0.0;
        for (int k = 0; k < desc->dim; k++) {
            double worst = 0.0;
            for (int lo = 0; lo < 4; lo++)
                for (int hi = 0; hi < 4; hi++) {
                    bool ok = true;
                    if ((lo == kFiner || hi == kFiner) && depth == desc->max_depth) ok = false;
                    if ((lo == kCoarser || hi == kCoarser) && depth == 0) ok = false;
                    if (lo == kBoundary && hi == kBoundary && !(depth == 0 && desc->n[k] == 1)) ok = false;
                    const bool sib_lo = lo == kSame || lo == kFiner, sib_hi = hi == kSame || hi == kFiner;
                    if (depth > 0 && !sib_lo && !sib_hi) ok = false;
                    if (ok) worst = std::max(worst, G[lo][hi]);
                }
            const double h = std::ldexp(desc->len[k] / (double)desc->n[k], -depth);
            s += C.Dk[k] / (h * h) * worst;
        }
        if (C.full) {
            // the worst admissible combination of the kinds of all faces
            double h0[3];
            for (int k = 0; k < 3; k++) h0[k] = k < desc->dim ? desc->len[k] / (double)desc->n[k] : 1.0;
            std::vector<double> tab;
            if (!own_block_table(R, desc->dim, h0, C, gamma, tab)) return MDLTS_EINVAL;
            double worst = 0.0;
            for (size_t idx = 0; idx < tab.size(); idx++) {
                bool ok = true;
                for (int k = 0; k < desc->dim && ok; k++) {
                    const uint32_t lo = (uint32_t)(idx >> (4 * k)) & 3, hi = (uint32_t)(idx >> (4 * k + 2)) & 3;
                    if ((lo == kFiner || hi == kFiner) && depth == desc->max_depth) ok = false;
                    if ((lo == kCoarser || hi == kCoarser) && depth == 0) ok = false;
                    if (lo == kBoundary && hi == kBoundary && !(depth == 0 && desc->n[k] == 1)) ok = false;
                    const bool sib_lo = lo == kSame || lo == kFiner, sib_hi = hi == kSame || hi == kFiner;
                    if (depth > 0 && !sib_lo && !sib_hi) ok = false;
                }
                if (ok) worst = std::max(worst, tab[idx]);
            }
            s = worst * std::ldexp(1.0, 2 * depth);
        }
        *cfl_min = 1.0 / s;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_plan_adapt(const mdlts_mesh_desc *desc, const uint8_t *bits, size_t n_bits, const double *eta,
                              size_t n_leaves, double tau_refine, double tau_coarsen, uint8_t *out_bits, size_t cap,
                              size_t *n_out)
{
    return abi_guard([&]() -> mdlts_status {
        if (!valid_desc(desc) || !eta || !n_out) return MDLTS_EINVAL;
        Forest F;
        forest_from_desc(desc, F);
        if (!F.parse_bits(bits, n_bits)) return MDLTS_EINVAL;
        if (F.size() != n_leaves) return MDLTS_EINVAL;
        AdaptPlan plan;
        if (!plan_adapt(F, eta, tau_refine, tau_coarsen, plan)) return MDLTS_EINVAL;
        std::vector<uint8_t> out;
        plan.next.write_bits(out);
        *n_out = out.size();
        if (out_bits && cap >= out.size()) std::memcpy(out_bits, out.data(), out.size());
        return MDLTS_OK;
    });
}

mdlts_status mdlts_memory_bound(const mdlts_mesh_desc *desc, int64_t max_leaves, uint64_t *bytes)
{
    return abi_guard([&]() -> mdlts_status {
        if (!valid_desc(desc) || max_leaves < 1 || max_leaves >= (1 << 27) || !bytes) return MDLTS_EINVAL;
        const uint64_t d = (uint64_t)desc->dim;
        const uint64_t np = desc->dim == 2 ? (uint64_t)(desc->order + 1) * (desc->order + 1)
                                           : (uint64_t)(desc->order + 1) * (desc->order + 1) * (desc->order + 1);
        const uint64_t T = desc->precision == MDLTS_FP64 ? 8 : 4;
        const uint64_t ksz = desc->dim == 2 ? 4 : 8;
        const uint64_t ns = desc->dim == 2 ? 2 : 4;
        const uint64_t nsub = 1ull << (desc->n_levels - 1);
        // every buffer a simulation holds is sized by its largest leaf count
        const uint64_t per_leaf =
            9 * np * T                  // u and v canonical, transfer copies, two u slots and v grouped, RV-T snapshot
            + 8 * np                    // FP64 staging of uploads and readbacks
            + 3 * ksz + 4               // canonical, new and grouped keys; Morton keys
            + 2 * (2 * d * 4)           // face tables, canonical and grouped
            + 2 * (2 * d * ns * 4)      // sub-face tables, canonical and grouped
            + 1 + 1 + 4 + 4 + 4 + 1     // refine and coarsen flags, counts, offsets, root offsets, scan sums
            + 1 + 4 + 1                 // transfer kind, source and child
            + 1 + 8 + 4 + 4 + 8 + 8 + 1 // level, CFL, permutation both ways, indicators, histogram share
            + lanes_per_element(desc->dim, desc->order, false) * ((nsub * 16 + 31) / 32);
                                    // batch tiles: per substep one per 64 threads (blocks of >= 64)
        const uint64_t fixed = 64 * per_leaf    // grouped arrays padded to whole blocks of 64 elements
                               + 64 * 512       // allocator rounding of every buffer
                               + 4 * 4096       // flags, step constants, batch descriptor, small scans
                               + 8 * 4096       // own-block bounds of a full diffusion tensor
                               + nsub * 16 * 2; // tile list heads
        // every buffer may hold 1/8 growth headroom (dev_alloc)
        *bytes = (per_leaf + (per_leaf + 7) / 8) * (uint64_t)max_leaves + fixed + fixed / 8;
        return MDLTS_OK;
    });
}

mdlts_status mdlts_plan_levels(const mdlts_mesh_desc *desc, const uint8_t *bits, size_t n_bits, const double D_sym[6],
                               double gamma, double dt_barrier, int8_t *level, int32_t *perm, int32_t *cnt_ge,
                               double *cfl, size_t n_leaves)
{
    return abi_guard([&]() -> mdlts_status {
        if (!valid_desc(desc) || !(dt_barrier > 0.0) || !(gamma > 0.0)) return MDLTS_EINVAL;
        Conductivity C;
        if (!parse_conductivity(D_sym, desc->dim, C)) return MDLTS_EINVAL;
        Forest F;
        forest_from_desc(desc, F);
        if (!F.parse_bits(bits, n_bits)) return MDLTS_EINVAL;
        if (F.size() != n_leaves) return MDLTS_EINVAL;
        RefTables R;
        make_ref_tables(desc->order, R);
        double G[4][4];
        if (!gershgorin_table(R, gamma, G)) return MDLTS_EINVAL;
        double h0[3];
        for (int k = 0; k < 3; k++) h0[k] = k < desc->dim ? desc->len[k] / (double)desc->n[k] : 1.0;
        std::vector<double> c(n_leaves);
        if (C.full) {
            std::vector<double> tab;
            if (!own_block_table(R, desc->dim, h0, C, gamma, tab)) return MDLTS_EINVAL;
            host_cfl_full(F, tab, c.data());
        } else {
            host_cfl(F, h0, C.Dk, G, c.data());
        }
        std::vector<int> lv(n_leaves);
        mdlts_status st = MDLTS_OK;
        for (size_t e = 0; e < n_leaves; e++) {
            lv[e] = level_of(dt_barrier, c[e]);
            if (lv[e] > desc->n_levels - 1) st = MDLTS_EUNSTABLE;
        }
        if (cfl) std::memcpy(cfl, c.data(), n_leaves * sizeof(double));
        if (level)
            for (size_t e = 0; e < n_leaves; e++) level[e] = (int8_t)std::min(lv[e], 127);
        if (perm || cnt_ge) {
            size_t pos = 0;
            for (int l = desc->n_levels - 1; l >= 0; l--) {
                for (size_t e = 0; e < n_leaves; e++)
                    if (lv[e] == l) {
                        if (perm) perm[pos] = (int32_t)e;
                        pos++;
                    }
                if (cnt_ge) cnt_ge[l] = (int32_t)pos;
            }
        }
        return st;
    });
}

}  // extern "C"
