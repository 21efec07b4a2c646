// kernels.hpp -- device kernels of the SIPG-DG / synchronous-LTS hot path
// for gfx950 (64-wide wavefronts).  Included only by mdlts.hip.
//
// Layout in HBM (one simulation):
//   u      [2 slots][np][cap]  bulk precision T; element j of the level-grouped
//                              order, node n at u[slot*np*cap + n*cap + j]
//   v      [np][cap]           gate state (element-local, updated in place)
//   key    [cap]               packed depth + cell coordinates (2-D: 32 bit)
//   nbr    [2d][cap]           packed face entries: kind(2) | level(3) | id(27)
//                              (same-size or coarser neighbour)
//   fine   [2d][cap][2^(d-1)]  entries (level | id) of the finer neighbours
//                              of a face whose entry has kind "finer"
// Element threads read their own nodes with unit stride across the wave
// (coalesced), and gather neighbour nodes through the face entries.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "host.hpp"

namespace mdlts {

constexpr uint32_t kIdMask27 = 0x07ffffffu;
constexpr uint32_t kIdMask30 = 0x3fffffffu;
constexpr int kMaxStim = 8;
constexpr int kMaxLevels = 8;

// 1-D reference tables of degree p (Sec. 2.1: Lagrange basis at the p+1
// Gauss-Legendre nodes, quadrature on the same nodes), evaluated by the
// compiler so that the substep kernel carries them as instruction
// constants.  Same construction as the host tables (barycentric weights).
struct RefConst {
    int m;
    double xi[kMaxM], w[kMaxM], winv[kMaxM], lam[kMaxM];
    double D1[kMaxM][kMaxM];       // D1[a][b] = l_b'(xi_a)
    double A[kMaxM][kMaxM];        // (1/w_a) sum_q w_q D1[q][a] D1[q][b]
    double W1[kMaxM][kMaxM];       // w_q D1[q][a] / w_a: weak derivative, A = W1 D1
    double B[2][kMaxM];            // l_b(-1), l_b(+1)
    double G[2][kMaxM];            // l_b'(-1), l_b'(+1)
    double Isub[2][kMaxM][kMaxM];  // l_b((xi_g + 2 pos - 1) / 2)
    double Lsub[2][kMaxM][kMaxM];  // w_g Isub[pos][g][a] / (2 w_a)
};

constexpr double csqrt(double x)
{
    double r = x > 1.0 ? x : 1.0;
    for (int k = 0; k < 200; k++) {
        const double n = 0.5 * (r + x / r);
        if (n == r) break;
        r = n;
    }
    return r;
}

constexpr double clagrange(const RefConst &T, int b, double x)
{
    double v = T.lam[b];
    for (int k = 0; k < T.m; k++)
        if (k != b) v *= (x - T.xi[k]);
    return v;
}

constexpr double clagrange_deriv(const RefConst &T, int b, double x)
{
    double s = 0.0;
    for (int k = 0; k < T.m; k++) {
        if (k == b) continue;
        double v = T.lam[b];
        for (int q = 0; q < T.m; q++)
            if (q != b && q != k) v *= (x - T.xi[q]);
        s += v;
    }
    return s;
}

constexpr RefConst ref_const(int p)
{
    RefConst T{};
    if (p == 1) {
        T.m = 2;
        const double r = 1.0 / csqrt(3.0);
        T.xi[0] = -r; T.xi[1] = r;
        T.w[0] = 1.0; T.w[1] = 1.0;
    } else if (p == 2) {
        T.m = 3;
        const double r = csqrt(0.6);
        T.xi[0] = -r; T.xi[1] = 0.0; T.xi[2] = r;
        T.w[0] = 5.0 / 9.0; T.w[1] = 8.0 / 9.0; T.w[2] = 5.0 / 9.0;
    } else {
        // roots of P_4: x^2 = 3/7 -+ (2/7) sqrt(6/5); weights (18 +- sqrt(30))/36
        T.m = 4;
        const double a = csqrt(3.0 / 7.0 - 2.0 / 7.0 * csqrt(1.2));
        const double b = csqrt(3.0 / 7.0 + 2.0 / 7.0 * csqrt(1.2));
        T.xi[0] = -b; T.xi[1] = -a; T.xi[2] = a; T.xi[3] = b;
        const double wa = (18.0 + csqrt(30.0)) / 36.0, wb = (18.0 - csqrt(30.0)) / 36.0;
        T.w[0] = wb; T.w[1] = wa; T.w[2] = wa; T.w[3] = wb;
    }
    const int m = T.m;
    for (int j = 0; j < m; j++) {
        double d = 1.0;
        for (int k = 0; k < m; k++)
            if (k != j) d *= (T.xi[j] - T.xi[k]);
        T.lam[j] = 1.0 / d;
        T.winv[j] = 1.0 / T.w[j];
    }
    for (int a = 0; a < m; a++) {
        double diag = 0.0;
        for (int b = 0; b < m; b++) {
            if (a == b) continue;
            T.D1[a][b] = (T.lam[b] / T.lam[a]) / (T.xi[a] - T.xi[b]);
            diag -= T.D1[a][b];
        }
        T.D1[a][a] = diag;
    }
    for (int a = 0; a < m; a++)
        for (int b = 0; b < m; b++) {
            double s = 0.0;
            for (int q = 0; q < m; q++) s += T.w[q] * T.D1[q][a] * T.D1[q][b];
            T.A[a][b] = s / T.w[a];
            T.W1[a][b] = T.w[b] * T.D1[b][a] / T.w[a];
        }
    for (int s = 0; s < 2; s++)
        for (int b = 0; b < m; b++) {
            T.B[s][b] = clagrange(T, b, s ? 1.0 : -1.0);
            T.G[s][b] = clagrange_deriv(T, b, s ? 1.0 : -1.0);
        }
    for (int pos = 0; pos < 2; pos++)
        for (int g = 0; g < m; g++)
            for (int b = 0; b < m; b++) T.Isub[pos][g][b] = clagrange(T, b, 0.5 * (T.xi[g] + 2.0 * pos - 1.0));
    for (int pos = 0; pos < 2; pos++)
        for (int a = 0; a < m; a++)
            for (int g = 0; g < m; g++) T.Lsub[pos][a][g] = T.w[g] * T.Isub[pos][g][a] / (2.0 * T.w[a]);
    return T;
}

template <typename T>
struct DevRef {
    T A[kMaxM][kMaxM];
    T B[2][kMaxM], G[2][kMaxM];
    T Isub[2][kMaxM][kMaxM], Lsub[2][kMaxM][kMaxM];
    T w[kMaxM], winv[kMaxM];
    double xi[kMaxM];
};

// Per-assignment constants of the substep kernel, kept in device memory
// (kernel arguments carry only the per-launch values below).
template <typename T>
struct StepArgs {
    long long slot_stride;
    uint32_t slot_bytes;  // slot_stride * sizeof(T); both slots fit in 4 GiB
    uint32_t node_bytes;  // cap * sizeof(T)
    int cap;
    int lmax;
    int cnt_ge[kMaxLevels];
    double dt_bar;
    double h0[3];
    T inv_h0[3];  // 1/h of a root; 1/h at depth d is inv_h0 * 2^d (exact)
    T Dk[3];
    T Dx[3];   // off-diagonal Dxy, Dxz, Dyz
    int full;  // some off-diagonal entry is nonzero
    T gamma;
    T apk, apa, eps0, mu1, mu2;
    int n_stim;  // all boxes; the kernel checks their time windows
    double stim[kMaxStim][9];
    DevRef<T> ref;
};

// Per-launch kernel arguments (passed by value, so the data pointers are
// known to address global memory).
template <typename T>
struct StepLaunch {
    T *u;
    T *v;
    const void *key;
    const uint32_t *nbr;
    const uint32_t *fine;
    uint32_t node_bytes;  // cap * sizeof(T) (u and v are in the grouped layout, grp_elem)
    uint32_t slot_bytes;  // np * cap * sizeof(T): stride between the two u slots
    int cap;              // elements per table column
    int lmax;             // finest level present
    int i;                // substep index in the barrier interval
    int n_act;            // active prefix
    int parity;           // barriers since the level assignment, mod 2
    double t_i;           // substep start time
};

template <int DIM>
struct KeyOf;
template <>
struct KeyOf<2> {
    using type = uint32_t;
    static constexpr int bits = 14;
};
template <>
struct KeyOf<3> {
    using type = uint64_t;
    static constexpr int bits = 20;
};

template <int DIM>
__host__ __device__ inline typename KeyOf<DIM>::type pack_key(int depth, const uint32_t *c)
{
    using K = typename KeyOf<DIM>::type;
    constexpr int b = KeyOf<DIM>::bits;
    K k = (K)depth;
    for (int q = 0; q < DIM; q++) k |= (K)c[q] << (4 + b * q);
    return k;
}

template <int DIM>
__device__ __forceinline__ void unpack_key(typename KeyOf<DIM>::type k, int &depth, uint32_t *c)
{
    constexpr int b = KeyOf<DIM>::bits;
    depth = (int)(k & 15);
#pragma unroll
    for (int q = 0; q < DIM; q++) c[q] = (uint32_t)((k >> (4 + b * q)) & ((1u << b) - 1));
}

template <int DIM, int P>
struct Shape {
    static constexpr int M = P + 1;
    static constexpr int NP = DIM == 2 ? M * M : M * M * M;
    static constexpr int NF = DIM == 2 ? M : M * M;
    static constexpr int NS = DIM == 2 ? 2 : 4;
};

// node index of tangential point g and normal index b for faces normal to k
template <int DIM, int M>
__device__ __forceinline__ constexpr int fnode(int k, int g, int b)
{
    if (DIM == 2) return k == 0 ? b + M * g : g + M * b;
    const int g0 = g % M, g1 = g / M;
    if (k == 0) return b + M * (g0 + M * g1);
    if (k == 1) return g0 + M * (b + M * g1);
    return g0 + M * (g1 + M * b);
}

// blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// range of elements so that neighbour gathers hit that XCD's L2
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    const int i = b >> 3;
    return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

// Arrays are read and written through raw buffer resources: a descriptor
// (scalar registers) holds the array's base and byte size, and each access
// adds a per-lane 32-bit byte offset and a uniform one (node or face
// stride), so no address arithmetic runs on the vector unit.  An offset past
// the end reads 0 and drops the write instead of touching other memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_of(const void *p, uint32_t bytes)
{
    // dword 3 of a gfx9 raw buffer descriptor: 32-bit data format, no swizzle
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

template <typename T>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T x)
{
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, x), r, (int)voff, (int)soff, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(HIP_vector_base<uint32_t, 2>::Native_vec_, x), r,
                                              (int)voff, (int)soff, 0);
}

// Grouped state layout (u in two slots, v) of elements of np nodes: blocks
// of 64 elements, [node][element] inside a block, so that a wave's loads of
// its elements' nodes fall in one block of np * 64 values (the memory system
// streams them faster than np arrays of cap values: measured 5.6 against
// 5.1 TB/s for np = 27).  Q1 quadrilaterals (np = 4), whose launches are
// cache-resident and latency-bound, keep [node][cap] (the block arithmetic
// cost them 1 % per launch).  Byte offset of element j inside a slot:
template <typename T, int NP>
__host__ __device__ constexpr uint32_t grp_elem(uint32_t j)
{
    if (NP == 4) return j * (uint32_t)sizeof(T);
    return (j >> 6) * (uint32_t)(NP * 64 * sizeof(T)) + (j & 63u) * (uint32_t)sizeof(T);
}
// and the byte stride between an element's nodes (node_bytes = cap * sizeof(T))
template <typename T, int NP>
__host__ __device__ constexpr uint32_t grp_node(uint32_t node_bytes)
{
    return NP == 4 ? node_bytes : 64u * (uint32_t)sizeof(T);
}

// out = (I[pos0] (x) I[pos1]) in over the tangential points of a face
template <typename T, int DIM, int M>
__device__ __forceinline__ void tang_apply(const double (&I)[2][kMaxM][kMaxM], int pos0, int pos1, const T *in,
                                           T *out)
{
    if constexpr (DIM == 2) {
#pragma unroll
        for (int g = 0; g < M; g++) {
            T s = 0;
#pragma unroll
            for (int q = 0; q < M; q++) s += (pos0 ? (T)I[1][g][q] : (T)I[0][g][q]) * in[q];
            out[g] = s;
        }
    } else {
        T tmp[M * M];
#pragma unroll
        for (int g1 = 0; g1 < M; g1++)
#pragma unroll
            for (int g0 = 0; g0 < M; g0++) {
                T s = 0;
#pragma unroll
                for (int q = 0; q < M; q++) s += (pos0 ? (T)I[1][g0][q] : (T)I[0][g0][q]) * in[q + M * g1];
                tmp[g0 + M * g1] = s;
            }
#pragma unroll
        for (int g1 = 0; g1 < M; g1++)
#pragma unroll
            for (int g0 = 0; g0 < M; g0++) {
                T s = 0;
#pragma unroll
                for (int q = 0; q < M; q++) s += (pos1 ? (T)I[1][g1][q] : (T)I[0][g1][q]) * tmp[g0 + M * q];
                out[g0 + M * g1] = s;
            }
    }
}

// point g of tang_apply(I, pos0, pos1, in), in the same order of operations
template <typename T, int DIM, int M>
__device__ __forceinline__ T tang_point(const double (&I)[2][kMaxM][kMaxM], int pos0, int pos1, const T *in, int g)
{
    if constexpr (DIM == 2) {
        T s = 0;
#pragma unroll
        for (int q = 0; q < M; q++) s += (pos0 ? (T)I[1][g][q] : (T)I[0][g][q]) * in[q];
        return s;
    } else {
        const int g0 = g % M, g1 = g / M;
        T s = 0;
#pragma unroll
        for (int q1 = 0; q1 < M; q1++) {
            T t = 0;
#pragma unroll
            for (int q = 0; q < M; q++) t += (pos0 ? (T)I[1][g0][q] : (T)I[0][g0][q]) * in[q + M * q1];
            s += (pos1 ? (T)I[1][g1][q1] : (T)I[0][g1][q1]) * t;
        }
        return s;
    }
}

// out = Op applied along direction k of an element array (lines of M nodes)
template <typename T, int DIM, int M>
__device__ __forceinline__ void line_apply(const double (&Op)[kMaxM][kMaxM], int k, const T *in, T *out)
{
    constexpr int NF = DIM == 2 ? M : M * M;
#pragma unroll
    for (int g = 0; g < NF; g++)
#pragma unroll
        for (int aa = 0; aa < M; aa++) {
            T s = 0;
#pragma unroll
            for (int b = 0; b < M; b++) s += (T)Op[aa][b] * in[fnode<DIM, M>(k, g, b)];
            out[fnode<DIM, M>(k, g, aa)] = s;
        }
}

// out = Op applied along tangential axis tau (0: g0, 1: g1) of a face array
// of points g0 + M g1
template <typename T, int DIM, int M>
__device__ __forceinline__ void face_line(const double (&Op)[kMaxM][kMaxM], int tau, const T *in, T *out)
{
    constexpr int NF = DIM == 2 ? M : M * M;
#pragma unroll
    for (int g = 0; g < NF; g++) {
        const int g0 = g % M, g1 = g / M;
        T s = 0;
#pragma unroll
        for (int c = 0; c < M; c++) s += (T)Op[tau ? g1 : g0][c] * in[tau ? g0 + M * c : c + M * g1];
        out[g] = s;
    }
}

// the direction of tangential axis tau of a face normal to k, and the slot
// of D_kt among the off-diagonal entries (xy, xz, yz)
__device__ __forceinline__ constexpr int tang_dir(int k, int tau) { return tau + (tau >= k ? 1 : 0); }
__device__ __forceinline__ constexpr int off_slot(int k, int t) { return k + t - 1; }

// Trace (value and reference normal derivative) of a neighbour on its face
// `side` normal to k, at the neighbour's interpolated time for substep i:
// a neighbour updated at this substep is read from its current slot; one
// that is not (it is coarser) is linear in time between its two slots.
template <typename T, int DIM, int P>
__device__ __forceinline__ void neighbour_trace(const StepArgs<T> &a, const StepLaunch<T> &L,
                                                __amdgpu_buffer_rsrc_t ru, uint32_t ent, int k, int side, T *tu,
                                                T *tq)
{
    const int si = L.i, parity = L.parity;
    using S = Shape<DIM, P>;
    constexpr int M = S::M;
    constexpr RefConst R = ref_const(P);
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = L.lmax - ln;
    const int base = ln == 0 ? parity : 0;
    const int cur = base ^ ((si >> sh) & 1);
    const int rem = si & ((1 << sh) - 1);
    const uint32_t o0 = (uint32_t)cur * L.slot_bytes + grp_elem<T, S::NP>(id);
#pragma unroll
    for (int g = 0; g < S::NF; g++) { tu[g] = 0; tq[g] = 0; }
    if (rem == 0) {
#pragma unroll
        for (int g = 0; g < S::NF; g++)
#pragma unroll
            for (int b = 0; b < M; b++) {
                const T val = buf_ld<T>(ru, o0, (uint32_t)fnode<DIM, M>(k, g, b) * grp_node<T, S::NP>(L.node_bytes));
                tu[g] += (T)R.B[side][b] * val;
                tq[g] += (T)R.G[side][b] * val;
            }
    } else {
        const T th = ldexp((T)rem, -sh);
        const uint32_t o1 = (uint32_t)(cur ^ 1) * L.slot_bytes + grp_elem<T, S::NP>(id);
#pragma unroll
        for (int g = 0; g < S::NF; g++)
#pragma unroll
            for (int b = 0; b < M; b++) {
                const uint32_t so = (uint32_t)fnode<DIM, M>(k, g, b) * grp_node<T, S::NP>(L.node_bytes);
                const T val = ((T)1 - th) * buf_ld<T>(ru, o0, so) + th * buf_ld<T>(ru, o1, so);
                tu[g] += (T)R.B[side][b] * val;
                tq[g] += (T)R.G[side][b] * val;
            }
    }
}

// Value of a neighbour's nodes at substep i (packed entry: level | id): a
// neighbour updated at this substep is read from its current slot; one that
// is not (it is coarser) is linear in time between its two slots.  Both
// slots are always loaded (the second from the first's address when not
// needed), so that the loads of all faces of a small element issue together
// without branches and the wave waits for memory once.
template <typename T, int NP>
__device__ __forceinline__ void neighbour_values(const StepLaunch<T> &L, __amdgpu_buffer_rsrc_t ru, uint32_t ent,
                                                 T *val)
{
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = L.lmax - ln;
    const int cur = (ln == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const int rem = L.i & ((1 << sh) - 1);
    const T th = ldexp((T)rem, -sh);
    const uint32_t o0 = (uint32_t)cur * L.slot_bytes + grp_elem<T, NP>(id);
    const uint32_t o1 = rem ? (uint32_t)(cur ^ 1) * L.slot_bytes + grp_elem<T, NP>(id) : o0;
#pragma unroll
    for (int n = 0; n < NP; n++) {
        const T x0 = buf_ld<T>(ru, o0, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
        const T x1 = buf_ld<T>(ru, o1, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
        val[n] = x0 + th * (x1 - x0);
    }
}

// The two halves of neighbour_values for software pipelining: the current
// slot's values, then (at use) the interpolation towards the other slot for
// lanes whose neighbour is coarser and not updated at this substep.
template <typename T, int NP>
__device__ __forceinline__ void neighbour_slot0(const StepLaunch<T> &L, __amdgpu_buffer_rsrc_t ru, uint32_t ent,
                                                T *val)
{
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = L.lmax - ln;
    const int cur = (ln == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const uint32_t o0 = (uint32_t)cur * L.slot_bytes + grp_elem<T, NP>(id);
#pragma unroll
    for (int n = 0; n < NP; n++) val[n] = buf_ld<T>(ru, o0, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
}

template <typename T, int NP>
__device__ __forceinline__ void neighbour_interp(const StepLaunch<T> &L, __amdgpu_buffer_rsrc_t ru, uint32_t ent,
                                                 T *val)
{
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = L.lmax - ln;
    const int cur = (ln == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const int rem = L.i & ((1 << sh) - 1);
    if (rem) {
        const T th = ldexp((T)rem, -sh);
        const uint32_t o1 = (uint32_t)(cur ^ 1) * L.slot_bytes + grp_elem<T, NP>(id);
#pragma unroll
        for (int n = 0; n < NP; n++) {
            const T x1 = buf_ld<T>(ru, o1, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
            val[n] = val[n] + th * (x1 - val[n]);
        }
    }
}

// One substep (Sec. 2.3, Algorithm 1) for the active prefix of the
// level-grouped elements: element-volume diffusion, SIPG face fluxes
// (Sec. 2.1), inverse diagonal mass, Aliev-Panfilov reaction + stimulus,
// forward Euler for u and an exponential step for v.  Reads the current
// slot, writes the other one; v is updated in place.
//
// Memory schedule: Q1 quadrilaterals load their own nodes, face entries
// and (for same-size or coarser faces) one neighbour per face before any
// arithmetic, so a wave waits for memory twice: their launches are short and
// latency-bound.  Larger elements keep one face's neighbour in flight while
// the previous face is computed, which leaves registers for more waves per
// SIMD (with the other register savings below: Q2 hexahedra 220 VGPRs and 2
// waves per SIMD, against 258 and 1 with two faces in flight; Q1 hexahedra
// 114 and 4).  Faces with finer neighbours (rare, at refinement interfaces)
// load their 2^(d-1) neighbours on demand.
// Large FP32 elements stage the gate v through LDS: its loads go straight
// to LDS at the start (no registers held) and are read at the update.
template <int DIM, int P, typename T>
constexpr bool kGateInLds = Shape<DIM, P>::NP > 16 && sizeof(T) == 4;

// ---- layouts of an element over the lanes ------------------------------------
// Q1 quadrilaterals with a diagonal tensor: four lanes per element (one node
// and one face each, substep_quad); every other element: one thread
// (substep_element).
__host__ __device__ constexpr bool uses_quad(int dim, int p, bool full) { return dim == 2 && p == 1 && !full; }
__host__ __device__ constexpr int node_count(int dim, int p)
{
    return dim == 2 ? (p + 1) * (p + 1) : (p + 1) * (p + 1) * (p + 1);
}
// elements per block of `block` threads (a multiple of 64)
__host__ __device__ constexpr int elements_per_block(int dim, int p, bool full, int block)
{
    return uses_quad(dim, p, full) ? block / 4 : block;
}

// Dynamic LDS of a launch: the gate staging area of per-thread elements above
// 16 nodes in FP32 (launches of fewer than 4 waves per block take less, so
// more blocks fit on a CU).  Same condition as kGateInLds.
inline size_t gate_lds_bytes(int dim, int p, bool fp32, int block)
{
    const int np = node_count(dim, p);
    return fp32 && np > 16 ? (size_t)(block / 64) * (size_t)np * 64 * sizeof(float) : 0;
}

// the dynamic LDS of every substep kernel (only the gate staging uses it)
extern __shared__ float gate_dyn[];

// FULL: the diffusion tensor has off-diagonal entries (separate kernels, so
// that the diagonal case keeps its register budget)
template <int DIM, int P, typename T, bool FULL>
__device__ __forceinline__ void substep_element(const StepArgs<T> &a, const StepLaunch<T> &L, const int j,
                                                const int lv, float *gate_lds)
{
    using S = Shape<DIM, P>;
    constexpr int M = S::M, NP = S::NP, NF = S::NF, NS = S::NS;
    constexpr int NFACE = 2 * DIM;
    // prefetch every face's neighbour: Q1 quadrilaterals only
    constexpr bool kPrefetch = NFACE * NP <= 16;

    constexpr RefConst R = ref_const(P);
    const int sh = L.lmax - lv;
    const int cur = (lv == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const T dt = (T)ldexp(a.dt_bar, -lv);
    const uint32_t self_ent = ((uint32_t)lv << 27) | (uint32_t)j;

    // ---- loads that depend on nothing but j
    using KT = typename KeyOf<DIM>::type;
    const uint32_t oj = (uint32_t)j * 4u;                   // 32-bit tables
    const uint32_t ojt = grp_elem<T, NP>((uint32_t)j);      // bulk arrays (grouped layout)
    const __amdgpu_buffer_rsrc_t ru = buf_of(L.u, 2u * L.slot_bytes);
    const __amdgpu_buffer_rsrc_t rv = buf_of(L.v, L.slot_bytes);
    const __amdgpu_buffer_rsrc_t rn = buf_of(L.nbr, (uint32_t)NFACE * (uint32_t)L.cap * 4u);
    uint32_t ent[NFACE];
#pragma unroll
    for (int f = 0; f < NFACE; f++) ent[f] = buf_ld<uint32_t>(rn, oj, (uint32_t)f * (uint32_t)L.cap * 4u);
    const KT kraw = buf_ld<KT>(buf_of(L.key, (uint32_t)L.cap * (uint32_t)sizeof(KT)), (uint32_t)j * sizeof(KT), 0);
    const uint32_t ou = (uint32_t)cur * L.slot_bytes + ojt;
    // the gate is needed only at the end; small elements load it with the
    // first round of loads, large ones after the face phase (registers)
    constexpr bool kEarlyV = NP <= 16;
    constexpr bool kLdsV = kGateInLds<DIM, P, T>;
    // this wave's slice of the gate staging area: [node][lane]
    float *gv = gate_lds + (threadIdx.x >> 6) * (NP * 64);
    T u[NP], vv[kEarlyV ? NP : 1];
#pragma unroll
    for (int n = 0; n < NP; n++) {
        u[n] = buf_ld<T>(ru, ou, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
        if constexpr (kEarlyV) vv[n] = buf_ld<T>(rv, ojt, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
        if constexpr (kLdsV)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, gv + n * 64, 4, ojt, (uint32_t)n * grp_node<T, NP>(L.node_bytes), 0, 0);
    }
    // ---- one neighbour per face (same-size or coarser), at the substep time
    T nb[kPrefetch ? NFACE : 1][NP];
    if constexpr (kPrefetch) {
#pragma unroll
        for (int f = 0; f < NFACE; f++) {
            const uint32_t kind = ent[f] >> 30;
            const bool one = kind == kSame || kind == kCoarser;
            neighbour_values<T, NP>(L, ru, one ? ent[f] : self_ent, nb[f]);
        }
    }

    int depth;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<DIM>(kraw, depth, c);
    T ih[DIM];  // 1/h_k of this element
#pragma unroll
    for (int k = 0; k < DIM; k++) ih[k] = ldexp(a.inv_h0[k], depth);

    T r[NP];
#pragma unroll
    for (int n = 0; n < NP; n++) r[n] = 0;

    // element volume: -(4 D_kk / h_k^2) A along each direction, with the
    // scale folded into this element's copy of A (one fused multiply-add
    // per term)
#pragma unroll
    for (int k = 0; k < DIM; k++) {
        const T ck = (T)4 * a.Dk[k] * ih[k] * ih[k];
        T cA[M][M];
#pragma unroll
        for (int aa = 0; aa < M; aa++)
#pragma unroll
            for (int b = 0; b < M; b++) cA[aa][b] = ck * (T)R.A[aa][b];
#pragma unroll
        for (int g = 0; g < NF; g++)
#pragma unroll
            for (int aa = 0; aa < M; aa++) {
                T &rn = r[fnode<DIM, M>(k, g, aa)];
#pragma unroll
                for (int b = 0; b < M; b++) rn -= cA[aa][b] * u[fnode<DIM, M>(k, g, b)];
            }
    }

    // off-diagonal D: -(4 D_kl / (h_k h_l)) (W1_k D1_l + W1_l D1_k) u per pair k < l
    if constexpr (FULL) {
#pragma unroll
        for (int k = 0; k < DIM; k++)
#pragma unroll
            for (int l = k + 1; l < DIM; l++) {
                const T ckl = (T)4 * a.Dx[off_slot(k, l)] * ih[k] * ih[l];
                T d1[NP], wd[NP];
                line_apply<T, DIM, M>(R.D1, l, u, d1);
                line_apply<T, DIM, M>(R.W1, k, d1, wd);
#pragma unroll
                for (int n = 0; n < NP; n++) r[n] -= ckl * wd[n];
                line_apply<T, DIM, M>(R.D1, k, u, d1);
                line_apply<T, DIM, M>(R.W1, l, d1, wd);
#pragma unroll
                for (int n = 0; n < NP; n++) r[n] -= ckl * wd[n];
            }
    }

    // interior faces.  Elements that do not prefetch every face keep NB
    // faces' neighbours in flight: face f+NB's loads are issued as soon as
    // face f is done, so memory overlaps the arithmetic.  NB = 2 in FP32 up
    // to degree 2 (Q2 hexahedra 249 VGPRs, still 2 waves per SIMD; alone,
    // 3.5 % faster than NB = 1 for Q2 hexahedra and 2-4 % for Q1
    // hexahedra); degree 3 and FP64 keep NB = 1 for their register budget.
    constexpr int NB = (sizeof(T) == 4 && P <= 2) ? 2 : 1;
    T nbuf[NB][kPrefetch ? 1 : NP];
    auto issue = [&](int f, T *dst) {
        const uint32_t kind = ent[f] >> 30;
        const bool one = kind == kSame || kind == kCoarser;
        neighbour_slot0<T, NP>(L, ru, one ? ent[f] : self_ent, dst);
        // The loads are used only inside the next faces' conditional blocks,
        // and the compiler would otherwise sink them into those blocks,
        // issuing them just before their use (no time in flight).  An empty
        // asm with a memory clobber keeps them here.
        asm volatile("" ::: "memory");
    };
    if constexpr (!kPrefetch) {
#pragma unroll
        for (int f = 0; f < NB; f++) issue(f, nbuf[f]);
    }
    // one call per face direction and side.  Degree 3 passes both as
    // compile-time constants: its loop is too large to unroll, and run-time
    // face indices would put the element arrays in scratch memory.  Lower
    // degrees unroll a plain loop (measured a few per cent faster there).
    auto face = [&](auto kc, auto sc) {
        const int k = kc;
        const int s = sc;
        const T c2 = (T)2 * ih[k];
        const T Dkk = a.Dk[k];
        const T pen = a.gamma * Dkk * ih[k];  // gamma D / h
        int pos0 = 0, pos1 = 0;  // own position inside a coarser neighbour's face
        {
            int t = 0;
#pragma unroll
            for (int q = 0; q < DIM; q++) {
                if (q == k) continue;
                if (t == 0) pos0 = c[q] & 1; else pos1 = c[q] & 1;
                t++;
            }
        }
        {
            const int f = 2 * k + s;
            const uint32_t kind = ent[f] >> 30;
            if (kind != kBoundary) {
            const T ns = s ? (T)1 : (T)-1;
            const T qs = ns * Dkk * c2;
            T tu[NF], tq[NF];
#pragma unroll
            for (int g = 0; g < NF; g++) {
                T su = 0, sq = 0;
#pragma unroll
                for (int b = 0; b < M; b++) {
                    su += (T)R.B[s][b] * u[fnode<DIM, M>(k, g, b)];
                    sq += (T)R.G[s][b] * u[fnode<DIM, M>(k, g, b)];
                }
                tu[g] = su;
                tq[g] = sq;
            }
            T Fl[NF], Hl[NF];
            if (kind != kFiner) {
                T nu[NF], nq[NF];
                auto trace_from = [&](const T *nv) {
#pragma unroll
                    for (int g = 0; g < NF; g++) {
                        T su = 0, sq = 0;
#pragma unroll
                        for (int b = 0; b < M; b++) {
                            su += (T)R.B[1 - s][b] * nv[fnode<DIM, M>(k, g, b)];
                            sq += (T)R.G[1 - s][b] * nv[fnode<DIM, M>(k, g, b)];
                        }
                        nu[g] = su;
                        nq[g] = sq;
                    }
                };
                if constexpr (kPrefetch) {
#pragma unroll
                    for (int g = 0; g < NF; g++) {
                        T su = 0, sq = 0;
#pragma unroll
                        for (int b = 0; b < M; b++) {
                            su += (T)R.B[1 - s][b] * nb[f][fnode<DIM, M>(k, g, b)];
                            sq += (T)R.G[1 - s][b] * nb[f][fnode<DIM, M>(k, g, b)];
                        }
                        nu[g] = su;
                        nq[g] = sq;
                    }
                } else {
                    neighbour_interp<T, NP>(L, ru, ent[f], nbuf[f % NB]);
                    trace_from(nbuf[f % NB]);
                }
                const bool co = kind == kCoarser;  // h_nbr = 2h
                if (kind == kCoarser) {
                    T iu[NF], iq[NF];
                    tang_apply<T, DIM, M>(R.Isub, pos0, pos1, nu, iu);
                    tang_apply<T, DIM, M>(R.Isub, pos0, pos1, nq, iq);
#pragma unroll
                    for (int g = 0; g < NF; g++) { nu[g] = iu[g]; nq[g] = iq[g]; }
                }
                // sigma = gamma 1/2 (D/h + D/h_nbr); n.D grad on the neighbour
                // scales by 2/h_nbr.  Fl and Hl are formed already scaled for
                // the lift (by c2 and by c2 qs): F = 1/2 (qs tq + qn nq) - sigma [u],
                // H = 1/2 [u].
                const T sigma = co ? (T)0.75 * pen : pen;
                const T qn = ns * Dkk * (co ? ih[k] : c2);
                const T cf_q = (T)0.5 * c2 * qs, cf_n = (T)0.5 * c2 * qn, cf_j = c2 * sigma;
                const T ch = (T)0.5 * c2 * qs;
#pragma unroll
                for (int g = 0; g < NF; g++) {
                    const T jmp = tu[g] - nu[g];
                    Fl[g] = cf_q * tq[g] + cf_n * nq[g] - cf_j * jmp;
                    Hl[g] = ch * jmp;
                }
                if constexpr (FULL) {
                    // tangential parts of n.D grad u on both sides (their
                    // mean) and of n.D grad l_i (against the jump), both
                    // lifted with c2 ns D_kt / h_t
                    T sm[NF], df[NF], t0[NF], t1[NF];
#pragma unroll
                    for (int g = 0; g < NF; g++) { sm[g] = tu[g] + nu[g]; df[g] = tu[g] - nu[g]; }
#pragma unroll
                    for (int tau = 0; tau < DIM - 1; tau++) {
                        const int t = tang_dir(k, tau);
                        const T cc = ns * c2 * a.Dx[off_slot(k, t)] * ih[t];
                        face_line<T, DIM, M>(R.D1, tau, sm, t0);
                        face_line<T, DIM, M>(R.W1, tau, df, t1);
#pragma unroll
                        for (int g = 0; g < NF; g++) Fl[g] += cc * (t0[g] + t1[g]);
                    }
                }
            } else {
                const T sigma = (T)1.5 * pen;           // h_nbr = h/2
                const T qn = ns * Dkk * (T)2 * c2;
                if constexpr (P >= 3) {
                    // degree 3: the own-side terms on the whole face (the
                    // sub-face restrictions of the own trace, lifted back,
                    // give it unchanged: sum over sub-faces of Lsub Isub = I)
                    // keep the reference tables out of scratch memory
                    // Own-side terms are taken on the whole face: restricting the
                    // own trace to the sub-faces (Isub) and lifting back (Lsub)
                    // gives it unchanged, since the half-interval GL rules
                    // integrate l_a l_b exactly (sum over sub-faces of Lsub Isub
                    // = I).  Only the neighbours' traces go through the sub-faces.
    #pragma unroll
                    for (int g = 0; g < NF; g++) {
                        Fl[g] = (T)0.5 * qs * tq[g] - sigma * tu[g];
                        Hl[g] = (T)0.5 * tu[g];
                    }
                    if constexpr (FULL) {
                        // own tangential derivatives (in face coordinates)
                        T t0[NF];
    #pragma unroll
                        for (int tau = 0; tau < DIM - 1; tau++) {
                            const int t = tang_dir(k, tau);
                            const T co = ns * a.Dx[off_slot(k, t)] * ih[t];
                            face_line<T, DIM, M>(R.D1, tau, tu, t0);
    #pragma unroll
                            for (int g = 0; g < NF; g++) Fl[g] += co * t0[g];
                        }
                    }
                    auto sub_face = [&](int sub) {
                        const int p0 = sub & 1, p1 = sub >> 1;
                        T nu[NF], nq[NF], G[NF], lg[NF];
                        const uint32_t fe = buf_ld<uint32_t>(buf_of(L.fine, (uint32_t)NFACE * (uint32_t)L.cap * NS * 4u),
                                                             (uint32_t)(j * NS + sub) * 4u,
                                                             (uint32_t)f * (uint32_t)L.cap * NS * 4u);
                        neighbour_trace<T, DIM, P>(a, L, ru, fe, k, 1 - s, nu, nq);
    #pragma unroll
                        for (int g = 0; g < NF; g++) G[g] = (T)0.5 * qn * nq[g] + sigma * nu[g];
                        if constexpr (FULL) {
                            // the neighbour's tangential derivatives on the
                            // sub-face (extent h_t / 2)
                            T t0[NF];
    #pragma unroll
                            for (int tau = 0; tau < DIM - 1; tau++) {
                                const int t = tang_dir(k, tau);
                                const T cf = (T)2 * ns * a.Dx[off_slot(k, t)] * ih[t];
                                face_line<T, DIM, M>(R.D1, tau, nu, t0);
    #pragma unroll
                                for (int g = 0; g < NF; g++) G[g] += cf * t0[g];
                            }
                        }
                        tang_apply<T, DIM, M>(R.Lsub, p0, p1, G, lg);
    #pragma unroll
                        for (int g = 0; g < NF; g++) { Fl[g] += lg[g]; G[g] = (T)-0.5 * nu[g]; }
                        tang_apply<T, DIM, M>(R.Lsub, p0, p1, G, lg);
    #pragma unroll
                        for (int g = 0; g < NF; g++) Hl[g] += lg[g];
                    };
                    if constexpr (NP <= 16) {
    #pragma unroll
                        for (int sub = 0; sub < NS; sub++) sub_face(sub);
                    } else {
    #pragma unroll 1
                        for (int sub = 0; sub < NS; sub++) sub_face(sub);
                    }
                } else {
    #pragma unroll
                    for (int g = 0; g < NF; g++) { Fl[g] = 0; Hl[g] = 0; }
                    // Per sub-face: the own trace restricted to its points (Isub),
                    // formed point by point (no arrays held), and the jump taken
                    // before any scaling, so that in FP32 the penalty multiplies a
                    // small difference; then both lifted back to the face (Lsub).
                    auto sub_face = [&](int sub) {
                        const int p0 = sub & 1, p1 = sub >> 1;
                        T nu[NF], nq[NF], G[NF], J[NF], lg[NF];
                        const uint32_t fe = buf_ld<uint32_t>(buf_of(L.fine, (uint32_t)NFACE * (uint32_t)L.cap * NS * 4u),
                                                             (uint32_t)(j * NS + sub) * 4u,
                                                             (uint32_t)f * (uint32_t)L.cap * NS * 4u);
                        neighbour_trace<T, DIM, P>(a, L, ru, fe, k, 1 - s, nu, nq);
    #pragma unroll
                        for (int g = 0; g < NF; g++) {
                            const T ou = tang_point<T, DIM, M>(R.Isub, p0, p1, tu, g);
                            const T oq = tang_point<T, DIM, M>(R.Isub, p0, p1, tq, g);
                            const T jmp = ou - nu[g];
                            G[g] = (T)0.5 * (qs * oq + qn * nq[g]) - sigma * jmp;
                            J[g] = (T)0.5 * jmp;
                        }
                        if constexpr (FULL) {
                            // tangential derivatives of both sides on the
                            // sub-face (extent h_t / 2)
                            T sm[NF], t0[NF];
                            tang_apply<T, DIM, M>(R.Isub, p0, p1, tu, sm);
    #pragma unroll
                            for (int g = 0; g < NF; g++) sm[g] += nu[g];
    #pragma unroll
                            for (int tau = 0; tau < DIM - 1; tau++) {
                                const int t = tang_dir(k, tau);
                                const T cf = (T)2 * ns * a.Dx[off_slot(k, t)] * ih[t];
                                face_line<T, DIM, M>(R.D1, tau, sm, t0);
    #pragma unroll
                                for (int g = 0; g < NF; g++) G[g] += cf * t0[g];
                            }
                        }
                        tang_apply<T, DIM, M>(R.Lsub, p0, p1, G, lg);
    #pragma unroll
                        for (int g = 0; g < NF; g++) Fl[g] += lg[g];
                        tang_apply<T, DIM, M>(R.Lsub, p0, p1, J, lg);
    #pragma unroll
                        for (int g = 0; g < NF; g++) Hl[g] += lg[g];
                    };
                    if constexpr (NP <= 16) {
    #pragma unroll
                        for (int sub = 0; sub < NS; sub++) sub_face(sub);
                    } else {
    #pragma unroll 1
                        for (int sub = 0; sub < NS; sub++) sub_face(sub);
                    }
                }
                if constexpr (FULL) {
                    // n.D grad l_i along the face against the lifted half
                    // jumps (Hl before its scaling)
                    T t1[NF];
#pragma unroll
                    for (int tau = 0; tau < DIM - 1; tau++) {
                        const int t = tang_dir(k, tau);
                        const T cj = (T)2 * ns * a.Dx[off_slot(k, t)] * ih[t];
                        face_line<T, DIM, M>(R.W1, tau, Hl, t1);
#pragma unroll
                        for (int g = 0; g < NF; g++) Fl[g] += cj * t1[g];
                    }
                }
                const T chq = c2 * qs;
#pragma unroll
                for (int g = 0; g < NF; g++) { Fl[g] *= c2; Hl[g] *= chq; }
            }
            // lift to the own nodes, already multiplied by the inverse mass:
            // r += c2 winv (F B + qs H G), with c2 and c2 qs already in Fl, Hl
            // (two fused multiply-adds into r per node)
#pragma unroll
            for (int g = 0; g < NF; g++)
#pragma unroll
                for (int b = 0; b < M; b++) {
                    T &rn = r[fnode<DIM, M>(k, g, b)];
                    rn += Fl[g] * (T)(R.winv[b] * R.B[s][b]);
                    rn += Hl[g] * (T)(R.winv[b] * R.G[s][b]);
                }
            }
            if constexpr (!kPrefetch)
                if (f + NB < NFACE) issue(f + NB, nbuf[f % NB]);
        }
    };
    if constexpr (P >= 3) {
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        face(I0{}, I0{});
        face(I0{}, I1{});
        face(I1{}, I0{});
        face(I1{}, I1{});
        if constexpr (DIM == 3) {
            face(I2{}, I0{});
            face(I2{}, I1{});
        }
    } else {
#pragma unroll
        for (int k = 0; k < DIM; k++)
#pragma unroll
            for (int s = 0; s < 2; s++) face(k, s);
    }

    // pointwise reaction, stimulus and update; the parameters are read
    // before the first store (the stores could alias them for the compiler)
    const uint32_t ouo = (uint32_t)(cur ^ 1) * L.slot_bytes + ojt;
    const T apk = a.apk, apa = a.apa, eps0 = a.eps0, mu1 = a.mu1, mu2 = a.mu2;
    const T apa1 = (T)1 + apa;
    const T ndt_l2e = -dt * (T)1.4426950408889634;  // -dt log2(e) (FP32 gate step)
    bool any = false;  // some stimulus box is on at t_i
    for (int b = 0; b < a.n_stim; b++) any = any || (L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7]);
    // Nodes lie inside the element's box [lo, lo + h] (also after rounding:
    // lo + f h with 0 < f < 1 rounds into [lo, fl(lo + h)]), so an element
    // whose box misses every active stimulus box tests no node.
    bool hit = false;
    if (any) {
        for (int b = 0; b < a.n_stim; b++) {
            bool h = L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7];
#pragma unroll
            for (int k = 0; k < DIM; k++) {
                const double hk = ldexp(a.h0[k], -depth);
                const double lo = (double)c[k] * hk;
                h = h && lo <= a.stim[b][3 + k] && lo + hk >= a.stim[b][k];
            }
            hit = hit || h;
        }
    }
#pragma unroll
    for (int n = 0; n < NP; n++) {
        const T un = u[n];
        T vn;
        if constexpr (kEarlyV) {
            vn = vv[n];
        } else if constexpr (kLdsV) {
            // the LDS writes of the staging loads complete with vmcnt, which
            // the compiler does not track for them: wait before the first read
            if (n == 0) __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
            vn = gv[n * 64 + (threadIdx.x & 63)];
        } else {
            vn = buf_ld<T>(rv, ojt, (uint32_t)n * grp_node<T, NP>(L.node_bytes));
        }
        const T au = apk * un;
        const T f = -au * (un - apa) * (un - (T)1) - un * vn;
        // (r + f) + stimulus; the stimulus sum only where a box is on
        T rf = r[n] + f;
        if (hit) {
            T stim = 0;
            double X[3];
            int nn = n;
#pragma unroll
            for (int k = 0; k < DIM; k++) {
                const double hk = ldexp(a.h0[k], -depth);
                const double lo = (double)c[k] * hk;
                X[k] = lo + 0.5 * (R.xi[nn % M] + 1.0) * hk;
                nn /= M;
            }
            for (int b = 0; b < a.n_stim; b++) {
                bool in = L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7];
#pragma unroll
                for (int k = 0; k < DIM; k++) in = in && X[k] >= a.stim[b][k] && X[k] <= a.stim[b][3 + k];
                if (in) stim += (T)a.stim[b][8];
            }
            rf += stim;
        }
        T den = un + mu2;
        den = den < (T)1e-6 ? (T)1e-6 : den;
        const T vinf = au * (apa1 - un);
        T decay;
        if constexpr (sizeof(T) == 4) {
            // FP32 bulk: hardware reciprocal (1 ulp) and base-2 exponential
            // of -eps dt log2(e), the scale taken once per element
            const T eps = eps0 + mu1 * (vn * __builtin_amdgcn_rcpf(den));
            decay = __builtin_amdgcn_exp2f(eps * ndt_l2e);
        } else {
            const T eps = eps0 + mu1 * vn / den;
            decay = exp(-eps * dt);
        }
        buf_st<T>(ru, ouo, (uint32_t)n * grp_node<T, NP>(L.node_bytes), un + dt * rf);
        buf_st<T>(rv, ojt, (uint32_t)n * grp_node<T, NP>(L.node_bytes), vinf + (vn - vinf) * decay);
    }
}

// ---- Q1 quadrilaterals: four lanes per element -------------------------------
// Threads per element of a kernel variant: Q1 quadrilaterals with a diagonal
// diffusion tensor spread an element over the four lanes of a quad (lane q
// owns node q for the volume term, the reaction and the stores, and face q,
// direction q >> 1 and side q & 1, for the neighbour gather and the flux);
// every other variant maps one element to one thread.
__host__ __device__ constexpr int lanes_per_element(int dim, int p, bool full)
{
    return uses_quad(dim, p, full) ? 4 : 1;
}

// quad_perm data movement inside each quad of lanes (DPP, no LDS): lane l
// receives the value of lane (PERM >> 2l) & 3 of its quad
template <int PERM>
__device__ __forceinline__ float quad_move(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), PERM, 0xf, 0xf, false));
}
template <int PERM>
__device__ __forceinline__ double quad_move(double x)
{
    const HIP_vector_base<int, 2>::Native_vec_ w = __builtin_bit_cast(HIP_vector_base<int, 2>::Native_vec_, x);
    HIP_vector_base<int, 2>::Native_vec_ r;
    r[0] = __builtin_amdgcn_update_dpp(0, w[0], PERM, 0xf, 0xf, false);
    r[1] = __builtin_amdgcn_update_dpp(0, w[1], PERM, 0xf, 0xf, false);
    return __builtin_bit_cast(double, r);
}
constexpr int kQuadBcast0 = 0x00, kQuadBcast1 = 0x55, kQuadBcast2 = 0xaa, kQuadBcast3 = 0xff;
constexpr int kQuadXor1 = 0xb1;  // lanes 1 0 3 2
constexpr int kQuadXor2 = 0x4e;  // lanes 2 3 0 1

// x[i] = the value of lane i of the quad, in every lane
template <typename T>
__device__ __forceinline__ void quad_gather(T v, T *x)
{
    x[0] = quad_move<kQuadBcast0>(v);
    x[1] = quad_move<kQuadBcast1>(v);
    x[2] = quad_move<kQuadBcast2>(v);
    x[3] = quad_move<kQuadBcast3>(v);
}

// the sum over the quad's lanes of c[q], returned to lane q (a two-step
// butterfly: pairs of nodes by bit 0 of the lane, then single nodes by bit 1)
template <typename T>
__device__ __forceinline__ T quad_reduce_scatter(const T *c, int q)
{
    const bool b0 = q & 1, b1 = q & 2;
    T keep0 = b0 ? c[1] : c[0], keep1 = b0 ? c[3] : c[2];
    const T send0 = b0 ? c[0] : c[1], send1 = b0 ? c[2] : c[3];
    keep0 += quad_move<kQuadXor1>(send0);
    keep1 += quad_move<kQuadXor1>(send1);
    T keep = b1 ? keep1 : keep0;
    const T send = b1 ? keep0 : keep1;
    keep += quad_move<kQuadXor2>(send);
    return keep;
}

// The four nodes of a Q1 quadrilateral at the substep time (packed entry:
// level | id), read with per-lane byte offsets: a neighbour updated at this
// substep from its current slot, a coarser one not updated linear in time
// between its two slots (the second read from the first's address when not
// needed, so that the loads issue without branches).
template <typename T>
__device__ __forceinline__ void quad_neighbour(const StepLaunch<T> &L, __amdgpu_buffer_rsrc_t ru, uint32_t ent,
                                               T *val)
{
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = L.lmax - ln;
    const int cur = (ln == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const int rem = L.i & ((1 << sh) - 1);
    const T th = ldexp((T)rem, -sh);
    const uint32_t o0 = (uint32_t)cur * L.slot_bytes + grp_elem<T, 4>(id);
    const uint32_t o1 = rem ? (uint32_t)(cur ^ 1) * L.slot_bytes + grp_elem<T, 4>(id) : o0;
    // the second slot only where some lane of the wave interpolates (a
    // wave-uniform branch; x0 + 0 (x1 - x0) = x0 for the others)
    if (__builtin_amdgcn_ballot_w64(rem != 0) != 0) {
        T x0[4], x1[4];
#pragma unroll
        for (int n = 0; n < 4; n++) {
            x0[n] = buf_ld<T>(ru, o0 + (uint32_t)n * grp_node<T, 4>(L.node_bytes), 0);
            x1[n] = buf_ld<T>(ru, o1 + (uint32_t)n * grp_node<T, 4>(L.node_bytes), 0);
        }
#pragma unroll
        for (int n = 0; n < 4; n++) val[n] = x0[n] + th * (x1[n] - x0[n]);
    } else {
#pragma unroll
        for (int n = 0; n < 4; n++) val[n] = buf_ld<T>(ru, o0 + (uint32_t)n * grp_node<T, 4>(L.node_bytes), 0);
    }
}

// One substep of Q1 quadrilateral j (diagonal D) on lane q of its quad: the
// same operator as substep_element (Sec. 2.1 volume and SIPG faces, inverse
// diagonal mass; Sec. 2.3 reaction, forward Euler for u, exponential step
// for the gate).  A face is handled in its own frame: the element's nodes
// are relabelled so that the face's normal line is the second index (a swap
// of nodes 1 and 2 for faces normal to y), which keeps every lane on the
// same instructions whatever its face.
template <typename T>
__device__ __forceinline__ void substep_quad(const StepArgs<T> &a, const StepLaunch<T> &L, const int j, const int lv,
                                             const int q)
{
    constexpr RefConst R = ref_const(1);
    const int k = q >> 1, s = q & 1;  // this lane's face: direction and side
    const int sh = L.lmax - lv;
    const int cur = (lv == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const T dt = (T)ldexp(a.dt_bar, -lv);

    // ---- loads: own node q (u, v), face entry q, key; then face q's neighbour
    const uint32_t ojt = grp_elem<T, 4>((uint32_t)j);
    const __amdgpu_buffer_rsrc_t ru = buf_of(L.u, 2u * L.slot_bytes);
    const __amdgpu_buffer_rsrc_t rv = buf_of(L.v, L.slot_bytes);
    const __amdgpu_buffer_rsrc_t rn = buf_of(L.nbr, 4u * (uint32_t)L.cap * 4u);
    const uint32_t ent = buf_ld<uint32_t>(rn, (uint32_t)j * 4u + (uint32_t)q * (uint32_t)L.cap * 4u, 0);
    const uint32_t kraw = buf_ld<uint32_t>(buf_of(L.key, (uint32_t)L.cap * 4u), (uint32_t)j * 4u, 0);
    const uint32_t ou = (uint32_t)cur * L.slot_bytes + ojt;
    const T uq = buf_ld<T>(ru, ou + (uint32_t)q * grp_node<T, 4>(L.node_bytes), 0);
    const T vq = buf_ld<T>(rv, ojt + (uint32_t)q * grp_node<T, 4>(L.node_bytes), 0);
    const uint32_t kind = ent >> 30;
    const bool one = kind == kSame || kind == kCoarser;
    T nv[4];
    quad_neighbour<T>(L, ru, one ? ent : (((uint32_t)lv << 27) | (uint32_t)j), nv);

    int depth;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<2>(kraw, depth, c);
    const T ih0 = ldexp(a.inv_h0[0], depth), ih1 = ldexp(a.inv_h0[1], depth);

    T u[4];
    quad_gather<T>(uq, u);

    // ---- volume term of node q: -(4 D_kk / h_k^2) A along both directions;
    // the line partner of node q is node q^1 along x and q^2 along y, and A
    // of the two symmetric Gauss nodes has equal diagonal (and off-diagonal)
    // entries
    static_assert(R.A[0][0] == R.A[1][1] && R.A[0][1] == R.A[1][0], "Q1 line operator");
    T rq;
    {
        const T c0 = (T)4 * a.Dk[0] * ih0 * ih0, c1 = (T)4 * a.Dk[1] * ih1 * ih1;
        const T ux = quad_move<kQuadXor1>(uq), uy = quad_move<kQuadXor2>(uq);
        const T sx = (T)R.A[0][0] * uq + (T)R.A[0][1] * ux;
        const T sy = (T)R.A[0][0] * uq + (T)R.A[0][1] * uy;
        rq = -(c0 * sx) - c1 * sy;
    }

    // ---- face q in its own frame: w[g][b] = node (tangential g, normal b)
    T cf[4] = {0, 0, 0, 0};  // this face's lift to nodes 0..3
    if (kind != kBoundary) {
        const T ihk = k ? ih1 : ih0;
        const T Dkk = k ? a.Dk[1] : a.Dk[0];
        const T c2 = (T)2 * ihk;
        const T pen = a.gamma * Dkk * ihk;
        const T ns = s ? (T)1 : (T)-1;
        const T qs = ns * Dkk * c2;
        const int pos0 = (int)(k ? c[0] : c[1]) & 1;  // own half of a coarser neighbour's face
        // own nodes in the face frame: swap nodes 1 and 2 for faces normal to y
        const T w00 = u[0], w01 = k ? u[2] : u[1], w10 = k ? u[1] : u[2], w11 = u[3];
        const T Bs0 = s ? (T)R.B[1][0] : (T)R.B[0][0], Bs1 = s ? (T)R.B[1][1] : (T)R.B[0][1];
        const T Gs0 = s ? (T)R.G[1][0] : (T)R.G[0][0], Gs1 = s ? (T)R.G[1][1] : (T)R.G[0][1];
        const T Bn0 = s ? (T)R.B[0][0] : (T)R.B[1][0], Bn1 = s ? (T)R.B[0][1] : (T)R.B[1][1];
        const T Gn0 = s ? (T)R.G[0][0] : (T)R.G[1][0], Gn1 = s ? (T)R.G[0][1] : (T)R.G[1][1];
        T tu[2], tq[2];
        tu[0] = Bs0 * w00 + Bs1 * w01;
        tu[1] = Bs0 * w10 + Bs1 * w11;
        tq[0] = Gs0 * w00 + Gs1 * w01;
        tq[1] = Gs0 * w10 + Gs1 * w11;
        T Fl[2], Hl[2];
        if (kind != kFiner) {
            const T n00 = nv[0], n01 = k ? nv[2] : nv[1], n10 = k ? nv[1] : nv[2], n11 = nv[3];
            T nu[2], nq[2];
            nu[0] = Bn0 * n00 + Bn1 * n01;
            nu[1] = Bn0 * n10 + Bn1 * n11;
            nq[0] = Gn0 * n00 + Gn1 * n01;
            nq[1] = Gn0 * n10 + Gn1 * n11;
            const bool co = kind == kCoarser;  // h_nbr = 2h: its trace at the own sub-face points
            if (co) {
                const T i00 = pos0 ? (T)R.Isub[1][0][0] : (T)R.Isub[0][0][0];
                const T i01 = pos0 ? (T)R.Isub[1][0][1] : (T)R.Isub[0][0][1];
                const T i10 = pos0 ? (T)R.Isub[1][1][0] : (T)R.Isub[0][1][0];
                const T i11 = pos0 ? (T)R.Isub[1][1][1] : (T)R.Isub[0][1][1];
                const T a0 = i00 * nu[0] + i01 * nu[1], a1 = i10 * nu[0] + i11 * nu[1];
                const T b0 = i00 * nq[0] + i01 * nq[1], b1 = i10 * nq[0] + i11 * nq[1];
                nu[0] = a0; nu[1] = a1; nq[0] = b0; nq[1] = b1;
            }
            // F = 1/2 (qs tq + qn nq) - sigma [u], H = 1/2 [u], pre-scaled for the lift
            const T sigma = co ? (T)0.75 * pen : pen;
            const T qn = ns * Dkk * (co ? ihk : c2);
            const T cf_q = (T)0.5 * c2 * qs, cf_n = (T)0.5 * c2 * qn, cf_j = c2 * sigma;
            const T ch = (T)0.5 * c2 * qs;
#pragma unroll
            for (int g = 0; g < 2; g++) {
                const T jmp = tu[g] - nu[g];
                Fl[g] = cf_q * tq[g] + cf_n * nq[g] - cf_j * jmp;
                Hl[g] = ch * jmp;
            }
        } else {
            // two finer neighbours, one per half of the face: the own trace
            // restricted to each half's points, the jump formed there, both
            // lifted back to the face
            const T sigma = (T)1.5 * pen;  // h_nbr = h/2
            const T qn = ns * Dkk * (T)2 * c2;
            Fl[0] = Fl[1] = Hl[0] = Hl[1] = 0;
            const __amdgpu_buffer_rsrc_t rf = buf_of(L.fine, 4u * (uint32_t)L.cap * 2u * 4u);
#pragma unroll 1
            for (int sub = 0; sub < 2; sub++) {
                const uint32_t fe = buf_ld<uint32_t>(rf, ((uint32_t)q * (uint32_t)L.cap * 2u + (uint32_t)j * 2u +
                                                          (uint32_t)sub) * 4u, 0);
                T fv[4];
                quad_neighbour<T>(L, ru, fe, fv);
                const T f00 = fv[0], f01 = k ? fv[2] : fv[1], f10 = k ? fv[1] : fv[2], f11 = fv[3];
                T nu[2], nq[2], G[2], J[2];
                nu[0] = Bn0 * f00 + Bn1 * f01;
                nu[1] = Bn0 * f10 + Bn1 * f11;
                nq[0] = Gn0 * f00 + Gn1 * f01;
                nq[1] = Gn0 * f10 + Gn1 * f11;
#pragma unroll
                for (int g = 0; g < 2; g++) {
                    const T i0 = sub ? (T)R.Isub[1][g][0] : (T)R.Isub[0][g][0];
                    const T i1 = sub ? (T)R.Isub[1][g][1] : (T)R.Isub[0][g][1];
                    const T ou_ = i0 * tu[0] + i1 * tu[1];
                    const T oq_ = i0 * tq[0] + i1 * tq[1];
                    const T jmp = ou_ - nu[g];
                    G[g] = (T)0.5 * (qs * oq_ + qn * nq[g]) - sigma * jmp;
                    J[g] = (T)0.5 * jmp;
                }
#pragma unroll
                for (int g = 0; g < 2; g++) {
                    const T l0 = sub ? (T)R.Lsub[1][g][0] : (T)R.Lsub[0][g][0];
                    const T l1 = sub ? (T)R.Lsub[1][g][1] : (T)R.Lsub[0][g][1];
                    Fl[g] += l0 * G[0] + l1 * G[1];
                    Hl[g] += l0 * J[0] + l1 * J[1];
                }
            }
            const T chq = c2 * qs;
#pragma unroll
            for (int g = 0; g < 2; g++) { Fl[g] *= c2; Hl[g] *= chq; }
        }
        // lift to the face-frame nodes (already times the inverse mass), then
        // back to node numbers
        const T e0 = (T)(R.winv[0] * R.B[0][0]), e1 = (T)(R.winv[1] * R.B[0][1]);
        const T d0 = (T)(R.winv[0] * R.G[0][0]), d1 = (T)(R.winv[1] * R.G[0][1]);
        const T E0 = (T)(R.winv[0] * R.B[1][0]), E1 = (T)(R.winv[1] * R.B[1][1]);
        const T D0 = (T)(R.winv[0] * R.G[1][0]), D1 = (T)(R.winv[1] * R.G[1][1]);
        const T lb0 = s ? E0 : e0, lb1 = s ? E1 : e1, lg0 = s ? D0 : d0, lg1 = s ? D1 : d1;
        const T z00 = Fl[0] * lb0 + Hl[0] * lg0, z01 = Fl[0] * lb1 + Hl[0] * lg1;
        const T z10 = Fl[1] * lb0 + Hl[1] * lg0, z11 = Fl[1] * lb1 + Hl[1] * lg1;
        cf[0] = z00;
        cf[1] = k ? z10 : z01;
        cf[2] = k ? z01 : z10;
        cf[3] = z11;
    }
    rq += quad_reduce_scatter<T>(cf, q);

    // ---- node q: reaction, stimulus, update
    const uint32_t ouo = (uint32_t)(cur ^ 1) * L.slot_bytes + ojt + (uint32_t)q * grp_node<T, 4>(L.node_bytes);
    const T apk = a.apk, apa = a.apa, eps0 = a.eps0, mu1 = a.mu1, mu2 = a.mu2;
    T stim = 0;
    bool on = false;  // some stimulus box is on at t_i (the same for every lane)
    for (int b = 0; b < a.n_stim; b++) on = on || (L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7]);
    if (on) {
        double X[2];
#pragma unroll
        for (int d = 0; d < 2; d++) {
            const double hk = ldexp(a.h0[d], -depth);
            const double xi = ((d ? q >> 1 : q & 1) ? R.xi[1] : R.xi[0]);
            X[d] = (double)c[d] * hk + 0.5 * (xi + 1.0) * hk;
        }
        for (int b = 0; b < a.n_stim; b++) {
            const bool in = L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7] && X[0] >= a.stim[b][0] &&
                            X[0] <= a.stim[b][3] && X[1] >= a.stim[b][1] && X[1] <= a.stim[b][4];
            if (in) stim += (T)a.stim[b][8];
        }
    }
    const T f = -apk * uq * (uq - apa) * (uq - (T)1) - uq * vq;
    T den = uq + mu2;
    den = den < (T)1e-6 ? (T)1e-6 : den;
    const T vinf = apk * uq * ((T)1 + apa - uq);
    T decay;
    if constexpr (sizeof(T) == 4) {
        const T eps = eps0 + mu1 * (vq * __builtin_amdgcn_rcpf(den));
        decay = __expf(-eps * dt);
    } else {
        const T eps = eps0 + mu1 * vq / den;
        decay = exp(-eps * dt);
    }
    buf_st<T>(ru, ouo, 0, uq + dt * (rq + f + stim));
    buf_st<T>(rv, ojt + (uint32_t)q * grp_node<T, 4>(L.node_bytes), 0, vinf + (vq - vinf) * decay);
}

// one simulation: element j of the active prefix [0, n_act)
template <int DIM, int P, typename T, bool FULL>
__global__ __launch_bounds__(256) void k_substep(const StepArgs<T> *__restrict__ cst, const StepLaunch<T> L)
{
    const StepArgs<T> &a = *cst;
    // elements are grouped finest level first
    auto lv_of = [&](int j) {
        int lv = 0;
#pragma unroll
        for (int l = 1; l < kMaxLevels; l++) lv += (j < a.cnt_ge[l]) ? 1 : 0;
        return lv;
    };
    const int t = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    const int j = t / lanes_per_element(DIM, P, FULL);
    if (j >= L.n_act) return;
    if constexpr (uses_quad(DIM, P, FULL)) substep_quad<T>(a, L, j, lv_of(j), t & 3);
    else substep_element<DIM, P, T, FULL>(a, L, j, lv_of(j), gate_dyn);
}

// ---- many simulations in one launch ------------------------------------------
// A tile is up to elements_per_block consecutive active elements of one
// simulation, all of one level.
struct BatchTile {
    // the simulation's arrays as byte offsets from the kernel's base pointer
    long long off_u, off_v, off_key, off_nbr, off_fine;
    int sim;
    int start;
    int count;
    int packed;           // level | parity << 4 | lmax << 8 (parity of the tile list's barrier)
    uint32_t node_bytes;  // as in StepLaunch
    uint32_t slot_bytes;
};
static_assert(sizeof(BatchTile) == 64, "one scalar load per tile");

// Everything a batched launch needs about one simulation.  Data locations
// are byte offsets from the kernel's base pointer so that the kernel derives
// them from a global-memory kernel argument.
template <typename T>
struct BatchSim {
    StepArgs<T> a;
    double t_start, h_tick;
};

// Barrier counter of a simulation in a batch.  Two copies alternate: the
// launches of a barrier read one, and the first substep's launch writes the
// next barrier's count into the other, so no launch writes what it reads.
// (Each copy has its own tile list, which carries the barrier's parity.)
struct BatchClock {
    long long n_bar;  // barriers since t_start
};

// Substep i of the barrier interval for every tile of the list, one tile
// per block.  Blocks are dealt round-robin to the 8 XCDs; block b takes tile
// b/8 of XCD b%8's contiguous range, so that neighbour gathers stay in one
// XCD's L2.  (A persistent form, blocks walking several tiles, held about 45
// more VGPRs live across its loop and was never the fastest shape.)
template <int DIM, int P, typename T, bool FULL>
__global__ __launch_bounds__(256) void k_substep_batch(const BatchSim<T> *__restrict__ sims,
                                                       const BatchTile *__restrict__ tiles, int n_tiles, int i,
                                                       char *base, const BatchClock *__restrict__ clk,
                                                       BatchClock *__restrict__ clk_next)
{
    const int x = blockIdx.x & 7;
    const int q = n_tiles >> 3, r = n_tiles & 7;
    const int t0 = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    const int t1 = t0 + q + (x < r ? 1 : 0);
    const int t = t0 + (int)(blockIdx.x >> 3);
    if (t >= t1) return;
    {
        // everything the first loads need comes with the tile, read as one
        // 64-byte value (a single scalar load)
        typedef int TileWords __attribute__((ext_vector_type(16)));
        const BatchTile tl = __builtin_bit_cast(BatchTile, *reinterpret_cast<const TileWords *>(tiles + t));
        const BatchClock ck = clk[tl.sim];
        // every simulation has a tile at start 0 in substep 0: it advances
        // the simulation's clock for the next barrier (after its own work,
        // so that the element loads do not wait for the clock)
        // this thread's element of the tile and its part of it
        const int slot = (int)threadIdx.x / lanes_per_element(DIM, P, FULL);
        const int part = (int)threadIdx.x & 3;
        const bool advance = i == 0 && tl.start == 0 && threadIdx.x == 0;
        if (slot >= tl.count) {
            if (advance) clk_next[tl.sim] = BatchClock{ck.n_bar + 1};
            return;
        }
        const BatchSim<T> &d = sims[tl.sim];
        StepLaunch<T> L;
        L.u = reinterpret_cast<T *>(base + tl.off_u);
        L.v = reinterpret_cast<T *>(base + tl.off_v);
        L.key = base + tl.off_key;
        L.nbr = reinterpret_cast<const uint32_t *>(base + tl.off_nbr);
        L.fine = reinterpret_cast<const uint32_t *>(base + tl.off_fine);
        L.node_bytes = tl.node_bytes;
        L.slot_bytes = tl.slot_bytes;
        L.cap = (int)(tl.node_bytes / (uint32_t)sizeof(T));
        L.lmax = (tl.packed >> 8) & 15;
        L.i = i;
        L.n_act = 0;
        L.parity = (tl.packed >> 4) & 1;
        // t = t_start + n dt + i h, rounded like the host (no contraction)
        L.t_i = __dadd_rn(__dadd_rn(d.t_start, __dmul_rn((double)ck.n_bar, d.a.dt_bar)), __dmul_rn((double)i, d.h_tick));
        if constexpr (uses_quad(DIM, P, FULL)) {
            substep_quad<T>(d.a, L, tl.start + slot, tl.packed & 15, part);
        } else {
            substep_element<DIM, P, T, FULL>(d.a, L, tl.start + slot, tl.packed & 15, gate_dyn);
        }
        if (advance) clk_next[tl.sim] = BatchClock{ck.n_bar + 1};
    }
}

}  // namespace mdlts
