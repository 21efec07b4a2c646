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

#include "host.hpp"

namespace mdlts {

constexpr uint32_t kIdMask27 = 0x07ffffffu;
constexpr uint32_t kIdMask30 = 0x3fffffffu;
constexpr int kMaxStim = 8;
constexpr int kMaxLevels = 8;

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
    int cap;
    int lmax;
    int cnt_ge[kMaxLevels];
    double dt_bar;
    double h0[3];
    T inv_h0[3];  // 1/h of a root; 1/h at depth d is inv_h0 * 2^d (exact)
    T Dk[3];
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
    int i;       // substep index in the barrier interval
    int n_act;   // active prefix
    int parity;  // barriers since the level assignment, mod 2
    double t_i;  // substep start time
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

// out = (I[pos0] (x) I[pos1]) in over the tangential points of a face
template <typename T, int DIM, int M>
__device__ __forceinline__ void tang_apply(const T (&I)[2][kMaxM][kMaxM], int pos0, int pos1, const T *in, T *out)
{
    if constexpr (DIM == 2) {
#pragma unroll
        for (int g = 0; g < M; g++) {
            T s = 0;
#pragma unroll
            for (int q = 0; q < M; q++) s += (pos0 ? I[1][g][q] : I[0][g][q]) * in[q];
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
                for (int q = 0; q < M; q++) s += (pos0 ? I[1][g0][q] : I[0][g0][q]) * in[q + M * g1];
                tmp[g0 + M * g1] = s;
            }
#pragma unroll
        for (int g1 = 0; g1 < M; g1++)
#pragma unroll
            for (int g0 = 0; g0 < M; g0++) {
                T s = 0;
#pragma unroll
                for (int q = 0; q < M; q++) s += (pos1 ? I[1][g1][q] : I[0][g1][q]) * tmp[g0 + M * q];
                out[g0 + M * g1] = s;
            }
    }
}

// Trace (value and reference normal derivative) of a neighbour on its face
// `side` normal to k, at the neighbour's interpolated time for substep i:
// a neighbour updated at this substep is read from its current slot; one
// that is not (it is coarser) is linear in time between its two slots.
template <typename T, int DIM, int P>
__device__ __forceinline__ void neighbour_trace(const StepArgs<T> &a, const StepLaunch<T> &L, uint32_t ent, int k,
                                                int side, T *tu, T *tq)
{
    const int si = L.i, parity = L.parity;
    using S = Shape<DIM, P>;
    constexpr int M = S::M;
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = a.lmax - ln;
    const int base = ln == 0 ? parity : 0;
    const int cur = base ^ ((si >> sh) & 1);
    const int rem = si & ((1 << sh) - 1);
    const T *p0 = L.u + (long long)cur * a.slot_stride + id;
#pragma unroll
    for (int g = 0; g < S::NF; g++) { tu[g] = 0; tq[g] = 0; }
    if (rem == 0) {
#pragma unroll
        for (int g = 0; g < S::NF; g++)
#pragma unroll
            for (int b = 0; b < M; b++) {
                const T val = p0[(long long)fnode<DIM, M>(k, g, b) * a.cap];
                tu[g] += a.ref.B[side][b] * val;
                tq[g] += a.ref.G[side][b] * val;
            }
    } else {
        const T th = ldexp((T)rem, -sh);
        const T *p1 = L.u + (long long)(cur ^ 1) * a.slot_stride + id;
#pragma unroll
        for (int g = 0; g < S::NF; g++)
#pragma unroll
            for (int b = 0; b < M; b++) {
                const long long o = (long long)fnode<DIM, M>(k, g, b) * a.cap;
                const T val = ((T)1 - th) * p0[o] + th * p1[o];
                tu[g] += a.ref.B[side][b] * val;
                tq[g] += a.ref.G[side][b] * val;
            }
    }
}

// Value of a neighbour's nodes at substep i (packed entry: level | id): a
// neighbour updated at this substep is read from its current slot; one that
// is not (it is coarser) is linear in time between its two slots.  Both
// slots are always loaded (the second from the first's address when not
// needed) so that the loads of all faces issue together without branches.
template <typename T, int NP>
__device__ __forceinline__ void neighbour_values(const StepArgs<T> &a, const StepLaunch<T> &L, uint32_t ent, T *val)
{
    const int si = L.i, parity = L.parity;
    const uint32_t id = ent & kIdMask27;
    const int ln = (int)((ent >> 27) & 7);
    const int sh = a.lmax - ln;
    const int base = ln == 0 ? parity : 0;
    const int cur = base ^ ((si >> sh) & 1);
    const int rem = si & ((1 << sh) - 1);
    const T th = ldexp((T)rem, -sh);
    const T *p0 = L.u + (long long)cur * a.slot_stride + id;
    const T *p1 = rem ? L.u + (long long)(cur ^ 1) * a.slot_stride + id : p0;
#pragma unroll
    for (int n = 0; n < NP; n++) {
        const T x0 = p0[(long long)n * a.cap];
        const T x1 = p1[(long long)n * a.cap];
        val[n] = x0 + th * (x1 - x0);
    }
}

// One substep (Sec. 2.3, Algorithm 1) for the active prefix of the
// level-grouped elements: element-volume diffusion, SIPG face fluxes
// (Sec. 2.1), inverse diagonal mass, Aliev-Panfilov reaction + stimulus,
// forward Euler for u and an exponential step for v.  Reads the current
// slot, writes the other one; v is updated in place.
//
// Memory schedule: the element's own nodes, its face entries and (for
// same-size or coarser faces) one neighbour per face are loaded before any
// arithmetic, so a wave waits for memory twice; faces with finer neighbours
// (rare, at refinement interfaces) load their 2^(d-1) neighbours on demand.
template <int DIM, int P, typename T>
__device__ __forceinline__ void substep_element(const StepArgs<T> &a, const StepLaunch<T> &L, const int j)
{
    using S = Shape<DIM, P>;
    constexpr int M = S::M, NP = S::NP, NF = S::NF, NS = S::NS;
    constexpr int NFACE = 2 * DIM;
    // prefetch every face's neighbour unless it costs too many registers
    constexpr bool kPrefetch = NFACE * NP <= 64;

    int lv = 0;
#pragma unroll
    for (int l = 1; l < kMaxLevels; l++) lv += (j < a.cnt_ge[l]) ? 1 : 0;
    const int sh = a.lmax - lv;
    const int cur = (lv == 0 ? L.parity : 0) ^ ((L.i >> sh) & 1);
    const T dt = (T)ldexp(a.dt_bar, -lv);
    const uint32_t self_ent = ((uint32_t)lv << 27) | (uint32_t)j;

    // ---- loads that depend on nothing but j
    uint32_t ent[NFACE];
#pragma unroll
    for (int f = 0; f < NFACE; f++) ent[f] = L.nbr[(long long)f * a.cap + j];
    const typename KeyOf<DIM>::type kraw = static_cast<const typename KeyOf<DIM>::type *>(L.key)[j];
    const T *uc = L.u + (long long)cur * a.slot_stride + j;
    T *vp = L.v + j;
    // the gate is needed only at the end; small elements load it with the
    // first round of loads, large ones after the face phase (registers)
    constexpr bool kEarlyV = NP <= 16;
    T u[NP], vv[kEarlyV ? NP : 1];
#pragma unroll
    for (int n = 0; n < NP; n++) {
        u[n] = uc[(long long)n * a.cap];
        if constexpr (kEarlyV) vv[n] = vp[(long long)n * a.cap];
    }
    // ---- one neighbour per face (same-size or coarser), at the substep time
    T nb[kPrefetch ? NFACE : 1][NP];
    if constexpr (kPrefetch) {
#pragma unroll
        for (int f = 0; f < NFACE; f++) {
            const uint32_t kind = ent[f] >> 30;
            const bool one = kind == kSame || kind == kCoarser;
            neighbour_values<T, NP>(a, L, one ? ent[f] : self_ent, nb[f]);
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

    // element volume: -(4 D_kk / h_k^2) A along each direction
#pragma unroll
    for (int k = 0; k < DIM; k++) {
        const T ck = (T)4 * a.Dk[k] * ih[k] * ih[k];
#pragma unroll
        for (int g = 0; g < NF; g++)
#pragma unroll
            for (int aa = 0; aa < M; aa++) {
                T s = 0;
#pragma unroll
                for (int b = 0; b < M; b++) s += a.ref.A[aa][b] * u[fnode<DIM, M>(k, g, b)];
                r[fnode<DIM, M>(k, g, aa)] -= ck * s;
            }
    }

    // interior faces
#pragma unroll
    for (int k = 0; k < DIM; k++) {
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
        // elements too large to prefetch every face load the two neighbours
        // of this direction together (one memory round trip per direction)
        T nbd[2][kPrefetch ? 1 : NP];
        if constexpr (!kPrefetch) {
#pragma unroll
            for (int s = 0; s < 2; s++) {
                const uint32_t kind = ent[2 * k + s] >> 30;
                const bool one = kind == kSame || kind == kCoarser;
                neighbour_values<T, NP>(a, L, one ? ent[2 * k + s] : self_ent, nbd[s]);
            }
        }
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const int f = 2 * k + s;
            const uint32_t kind = ent[f] >> 30;
            if (kind == kBoundary) continue;
            const T ns = s ? (T)1 : (T)-1;
            const T qs = ns * Dkk * c2;
            T tu[NF], tq[NF];
#pragma unroll
            for (int g = 0; g < NF; g++) {
                T su = 0, sq = 0;
#pragma unroll
                for (int b = 0; b < M; b++) {
                    su += a.ref.B[s][b] * u[fnode<DIM, M>(k, g, b)];
                    sq += a.ref.G[s][b] * u[fnode<DIM, M>(k, g, b)];
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
                            su += a.ref.B[1 - s][b] * nv[fnode<DIM, M>(k, g, b)];
                            sq += a.ref.G[1 - s][b] * nv[fnode<DIM, M>(k, g, b)];
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
                            su += a.ref.B[1 - s][b] * nb[f][fnode<DIM, M>(k, g, b)];
                            sq += a.ref.G[1 - s][b] * nb[f][fnode<DIM, M>(k, g, b)];
                        }
                        nu[g] = su;
                        nq[g] = sq;
                    }
                } else {
                    trace_from(nbd[s]);
                }
                const bool co = kind == kCoarser;  // h_nbr = 2h
                if (kind == kCoarser) {
                    T iu[NF], iq[NF];
                    tang_apply<T, DIM, M>(a.ref.Isub, pos0, pos1, nu, iu);
                    tang_apply<T, DIM, M>(a.ref.Isub, pos0, pos1, nq, iq);
#pragma unroll
                    for (int g = 0; g < NF; g++) { nu[g] = iu[g]; nq[g] = iq[g]; }
                }
                // sigma = gamma 1/2 (D/h + D/h_nbr); n.D grad on the neighbour scales by 2/h_nbr
                const T sigma = co ? (T)0.75 * pen : pen;
                const T qn = ns * Dkk * (co ? ih[k] : c2);
#pragma unroll
                for (int g = 0; g < NF; g++) {
                    const T jmp = tu[g] - nu[g];
                    Fl[g] = (T)0.5 * (qs * tq[g] + qn * nq[g]) - sigma * jmp;
                    Hl[g] = (T)0.5 * jmp;
                }
            } else {
                const T sigma = (T)1.5 * pen;           // h_nbr = h/2
                const T qn = ns * Dkk * (T)2 * c2;
#pragma unroll
                for (int g = 0; g < NF; g++) { Fl[g] = 0; Hl[g] = 0; }
                auto sub_face = [&](int sub) {
                    const int p0 = sub & 1, p1 = sub >> 1;
                    T ou[NF], oq[NF], nu[NF], nq[NF], F[NF], H[NF], lf[NF], lh[NF];
                    tang_apply<T, DIM, M>(a.ref.Isub, p0, p1, tu, ou);
                    tang_apply<T, DIM, M>(a.ref.Isub, p0, p1, tq, oq);
                    neighbour_trace<T, DIM, P>(a, L, L.fine[((long long)f * a.cap + j) * NS + sub], k, 1 - s, nu, nq);
#pragma unroll
                    for (int g = 0; g < NF; g++) {
                        const T jmp = ou[g] - nu[g];
                        F[g] = (T)0.5 * (qs * oq[g] + qn * nq[g]) - sigma * jmp;
                        H[g] = (T)0.5 * jmp;
                    }
                    tang_apply<T, DIM, M>(a.ref.Lsub, p0, p1, F, lf);
                    tang_apply<T, DIM, M>(a.ref.Lsub, p0, p1, H, lh);
#pragma unroll
                    for (int g = 0; g < NF; g++) { Fl[g] += lf[g]; Hl[g] += lh[g]; }
                };
                if constexpr (NP <= 16) {
#pragma unroll
                    for (int sub = 0; sub < NS; sub++) sub_face(sub);
                } else {
#pragma unroll 1
                    for (int sub = 0; sub < NS; sub++) sub_face(sub);
                }
            }
            // lift to the own nodes, already multiplied by the inverse mass
#pragma unroll
            for (int g = 0; g < NF; g++)
#pragma unroll
                for (int b = 0; b < M; b++)
                    r[fnode<DIM, M>(k, g, b)] += c2 * a.ref.winv[b] * (Fl[g] * a.ref.B[s][b] + Hl[g] * qs * a.ref.G[s][b]);
        }
    }

    // pointwise reaction, stimulus and update
    T *uo = L.u + (long long)(cur ^ 1) * a.slot_stride + j;
#pragma unroll
    for (int n = 0; n < NP; n++) {
        const T un = u[n];
        T vn;
        if constexpr (kEarlyV) vn = vv[n];
        else vn = vp[(long long)n * a.cap];
        T stim = 0;
        bool any = false;
        for (int b = 0; b < a.n_stim; b++) any = any || (L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7]);
        if (any) {
            double X[3];
            int nn = n;
#pragma unroll
            for (int k = 0; k < DIM; k++) {
                const double hk = ldexp(a.h0[k], -depth);
                const double lo = (double)c[k] * hk;
                X[k] = lo + 0.5 * (a.ref.xi[nn % M] + 1.0) * hk;
                nn /= M;
            }
            for (int b = 0; b < a.n_stim; b++) {
                bool in = L.t_i >= a.stim[b][6] && L.t_i < a.stim[b][7];
#pragma unroll
                for (int k = 0; k < DIM; k++) in = in && X[k] >= a.stim[b][k] && X[k] <= a.stim[b][3 + k];
                if (in) stim += (T)a.stim[b][8];
            }
        }
        const T f = -a.apk * un * (un - a.apa) * (un - (T)1) - un * vn;
        T den = un + a.mu2;
        den = den < (T)1e-6 ? (T)1e-6 : den;
        const T vinf = a.apk * un * ((T)1 + a.apa - un);
        T decay;
        if constexpr (sizeof(T) == 4) {
            // FP32 bulk: fast reciprocal division and exponential
            const T eps = a.eps0 + a.mu1 * __fdividef(vn, den);
            decay = __expf(-eps * dt);
        } else {
            const T eps = a.eps0 + a.mu1 * vn / den;
            decay = exp(-eps * dt);
        }
        uo[(long long)n * a.cap] = un + dt * (r[n] + f + stim);
        vp[(long long)n * a.cap] = vinf + (vn - vinf) * decay;
    }
}

// one simulation: element j of the active prefix [0, n_act)
template <int DIM, int P, typename T>
__global__ __launch_bounds__(256) void k_substep(const StepArgs<T> *__restrict__ cst, const StepLaunch<T> L)
{
    const int j = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (j >= L.n_act) return;
    substep_element<DIM, P, T>(*cst, L, j);
}

// ---- many simulations in one launch ------------------------------------------
// A tile is up to blockDim.x consecutive active elements of one simulation.
struct BatchTile {
    int sim;
    int start;
    int count;
    int pad;
};

// Everything a batched launch needs about one simulation.  Data locations
// are byte offsets from the kernel's base pointer so that the kernel derives
// them from a global-memory kernel argument.
template <typename T>
struct BatchSim {
    StepArgs<T> a;
    long long off_u, off_v, off_key, off_nbr, off_fine;
    double t_start, h_tick;
    long long n_bar;  // barriers since t_start (advanced on the device)
    int parity;       // barriers since the level assignment, mod 2
    int pad;
};

// Substep i of the barrier interval for every tile of the list.  With a
// grid smaller than the tile count each block walks the tiles of its XCD's
// contiguous range (persistent form).
template <int DIM, int P, typename T>
__global__ __launch_bounds__(256) void k_substep_batch(const BatchSim<T> *__restrict__ sims,
                                                       const BatchTile *__restrict__ tiles, int n_tiles, int i,
                                                       char *base)
{
    const int x = blockIdx.x & 7, per = (int)(gridDim.x >> 3);
    const int q = n_tiles >> 3, r = n_tiles & 7;
    const int t0 = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    const int t1 = t0 + q + (x < r ? 1 : 0);
    for (int t = t0 + (int)(blockIdx.x >> 3); t < t1; t += per) {
        const BatchTile tl = tiles[t];
        if ((int)threadIdx.x >= tl.count) continue;
        const BatchSim<T> &d = sims[tl.sim];
        StepLaunch<T> L;
        L.u = reinterpret_cast<T *>(base + d.off_u);
        L.v = reinterpret_cast<T *>(base + d.off_v);
        L.key = base + d.off_key;
        L.nbr = reinterpret_cast<const uint32_t *>(base + d.off_nbr);
        L.fine = reinterpret_cast<const uint32_t *>(base + d.off_fine);
        L.i = i;
        L.n_act = 0;
        L.parity = d.parity;
        // t = t_start + n dt + i h, rounded like the host (no contraction)
        L.t_i = __dadd_rn(__dadd_rn(d.t_start, __dmul_rn((double)d.n_bar, d.a.dt_bar)), __dmul_rn((double)i, d.h_tick));
        substep_element<DIM, P, T>(d.a, L, tl.start + (int)threadIdx.x);
    }
}

// end of a barrier interval for every simulation of a batch
template <typename T>
__global__ void k_batch_advance(BatchSim<T> *sims, int n)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    sims[s].n_bar += 1;
    sims[s].parity ^= 1;
}

}  // namespace mdlts
