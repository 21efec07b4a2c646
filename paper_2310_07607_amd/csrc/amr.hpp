// amr.hpp -- device-resident mesh management: face tables from the leaf
// keys, and the adaptation step of Algorithm 1 (mark with the indicator,
// close the 2:1 balance, coarsen complete sibling groups, emit the new
// canonical leaf list).  Included only by mdlts.hip.
//
// Canonical device mesh:
//   key  [E]                depth | cell coordinates (pack_key)
//   face [2d][E]            kind << 30 | canonical neighbour (same / coarser)
//   fine [(f*E + e)*2^(d-1) + q]   the finer neighbours of face f of leaf e
// Leaves are in canonical order: roots in id order, pre-order inside a root,
// which is ascending Morton order of the lower corner at the depth cap.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"
#include "multi.hpp"

namespace mdlts {

struct MeshGeo {
    int n[3];
    int max_depth;
};

__device__ __forceinline__ uint32_t spread2_d(uint32_t x)
{
    x = (x | (x << 4)) & 0x0F0Fu;
    x = (x | (x << 2)) & 0x3333u;
    x = (x | (x << 1)) & 0x5555u;
    return x;
}

__device__ __forceinline__ uint32_t spread3_d(uint32_t x)
{
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

template <int DIM>
__device__ __forceinline__ int root_of(const MeshGeo &g, int depth, const uint32_t *c)
{
    int r = 0, mul = 1;
    for (int k = 0; k < DIM; k++) {
        r += (int)(c[k] >> depth) * mul;
        mul *= g.n[k];
    }
    return r;
}

// Morton key of the lower corner of cell c (level `depth`) inside its root
template <int DIM>
__device__ __forceinline__ uint32_t morton_in_root(const MeshGeo &g, int depth, const uint32_t *c)
{
    const int sh = g.max_depth - depth;
    uint32_t m = 0;
    for (int k = 0; k < DIM; k++) {
        const uint32_t loc = (c[k] & ((1u << depth) - 1u)) << sh;
        m |= (DIM == 2 ? spread2_d(loc) : spread3_d(loc)) << k;
    }
    return m;
}

// the leaf containing the lower corner of cell c at `depth`
template <int DIM>
__device__ __forceinline__ int find_containing(const MeshGeo &g, const int *root_start, const uint32_t *mkey, int depth,
                                               const uint32_t *c)
{
    const int r = root_of<DIM>(g, depth, c);
    const uint32_t m = morton_in_root<DIM>(g, depth, c);
    int lo = root_start[r];
    int len = root_start[r + 1] - lo;
    while (len > 1) {
        const int half = len >> 1;
        lo = mkey[lo + half] <= m ? lo + half : lo;
        len -= half;
    }
    return lo;
}

template <int DIM>
__device__ __forceinline__ void mesh_index_body(const int blk, int E, int n_roots, const MeshGeo g,
                                                    const typename KeyOf<DIM>::type *key, int *root_start,
                                                    uint32_t *mkey)
{
    const int e = blk * 256 + threadIdx.x;
    if (e >= E) return;
    int d;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<DIM>(key[e], d, c);
    mkey[e] = morton_in_root<DIM>(g, d, c);
    const int r = root_of<DIM>(g, d, c);
    bool first = e == 0;
    if (!first) {
        int dp;
        uint32_t cp[3] = {0, 0, 0};
        unpack_key<DIM>(key[e - 1], dp, cp);
        first = root_of<DIM>(g, dp, cp) != r;
    }
    if (first) root_start[r] = e;
    if (e == E - 1) root_start[n_roots] = E;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_mesh_index(int E, int n_roots, const MeshGeo g,
                                                    const typename KeyOf<DIM>::type *key, int *root_start,
                                                    uint32_t *mkey)
{
    mesh_index_body<DIM>(blockIdx.x, E, n_roots, g, key, root_start, mkey);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct MeshIndexOp {
    int E;
    int n_roots;
    MeshGeo g;
    const typename KeyOf<DIM>::type *key;
    int *root_start;
    uint32_t *mkey;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        mesh_index_body<DIM>(blk, E, n_roots, g, key, root_start, mkey);
    }
};

// face table of every leaf; *bad is set if the forest is not 2:1 balanced
template <int DIM>
__device__ __forceinline__ void mesh_faces_body(const int blk, int E, const MeshGeo g, const typename KeyOf<DIM>::type *key,
                                                    const int *root_start, const uint32_t *mkey, uint32_t *face,
                                                    uint32_t *fine, int *bad)
{
    constexpr int NS = DIM == 2 ? 2 : 4;
    // one thread per (face, element): face f = 2k + s of element e, elements
    // fastest, so that the key loads and the table stores are coalesced and
    // the faces' neighbour searches run side by side
    const long long i = (long long)blk * 256 + threadIdx.x;
    if (i >= 2ll * DIM * E) return;
    const int f = (int)(i / E);
    const int e = (int)(i - (long long)f * E);
    int d;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<DIM>(key[e], d, c);
    {
        const int k = f >> 1, s = f & 1;
        uint32_t t[3] = {c[0], c[1], c[2]};
        uint32_t entry = kBoundary << 30;
        const bool inside = s ? (c[k] + 1 < ((uint32_t)g.n[k] << d)) : (c[k] > 0);
        if (inside) {
            t[k] = s ? c[k] + 1 : c[k] - 1;
            const int id = find_containing<DIM>(g, root_start, mkey, d, t);
            int dn;
            uint32_t cn[3] = {0, 0, 0};
            unpack_key<DIM>(key[id], dn, cn);
            if (dn == d) {
                entry = (kSame << 30) | (uint32_t)id;
            } else if (dn + 1 == d) {
                entry = (kCoarser << 30) | (uint32_t)id;
            } else if (dn > d) {
                const int want = s ? 0 : 1;
                int q = 0;
                for (int ci = 0; ci < (1 << DIM); ci++) {
                    if (((ci >> k) & 1) != want) continue;
                    uint32_t cc[3] = {0, 0, 0};
                    for (int p = 0; p < DIM; p++) cc[p] = 2 * t[p] + ((ci >> p) & 1);
                    const int fid = find_containing<DIM>(g, root_start, mkey, d + 1, cc);
                    int df;
                    uint32_t cf[3];
                    unpack_key<DIM>(key[fid], df, cf);
                    if (df != d + 1) atomicOr(bad, 1);
                    fine[((long long)f * E + e) * NS + q] = (uint32_t)fid;
                    q++;
                }
                entry = kFiner << 30;
            } else {
                atomicOr(bad, 1);
            }
        }
        face[(long long)f * E + e] = entry;
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_mesh_faces(int E, const MeshGeo g, const typename KeyOf<DIM>::type *key,
                                                    const int *root_start, const uint32_t *mkey, uint32_t *face,
                                                    uint32_t *fine, int *bad)
{
    mesh_faces_body<DIM>(blockIdx.x, E, g, key, root_start, mkey, face, fine, bad);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct MeshFacesOp {
    int E;
    MeshGeo g;
    const typename KeyOf<DIM>::type *key;
    const int *root_start;
    const uint32_t *mkey;
    uint32_t *face;
    uint32_t *fine;
    int *bad;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        mesh_faces_body<DIM>(blk, E, g, key, root_start, mkey, face, fine, bad);
    }
};

// ---- adaptation ------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void amr_mark_body(const int blk, int E, const MeshGeo g, const typename KeyOf<DIM>::type *key,
                                                  const double *eta, double tau_refine, uint8_t *refine)
{
    const int e = blk * 256 + threadIdx.x;
    if (e >= E) return;
    const int d = (int)(key[e] & 15);
    refine[e] = (eta[e] >= tau_refine && d < g.max_depth) ? 1 : 0;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_amr_mark(int E, const MeshGeo g, const typename KeyOf<DIM>::type *key,
                                                  const double *eta, double tau_refine, uint8_t *refine)
{
    amr_mark_body<DIM>(blockIdx.x, E, g, key, eta, tau_refine, refine);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct AmrMarkOp {
    int E;
    MeshGeo g;
    const typename KeyOf<DIM>::type *key;
    const double *eta;
    double tau_refine;
    uint8_t *refine;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        amr_mark_body<DIM>(blk, E, g, key, eta, tau_refine, refine);
    }
};

// one pass of the 2:1 closure: a leaf being refined marks its coarser face
// neighbours (every chain of such marks descends one depth per step, so
// max_depth passes reach the least fixed point)
template <int DIM>
__device__ __forceinline__ void amr_close_body(const int blk, int E, const uint32_t *face, uint8_t *refine)
{
    const int e = blk * 256 + threadIdx.x;
    if (e >= E || !refine[e]) return;
    for (int f = 0; f < 2 * DIM; f++) {
        const uint32_t ent = face[(long long)f * E + e];
        if ((ent >> 30) == kCoarser) refine[ent & kIdMask30] = 1;
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_amr_close(int E, const uint32_t *face, uint8_t *refine)
{
    amr_close_body<DIM>(blockIdx.x, E, face, refine);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct AmrCloseOp {
    int E;
    const uint32_t *face;
    uint8_t *refine;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        amr_close_body<DIM>(blk, E, face, refine);
    }
};

template <int DIM>
__device__ __forceinline__ bool sibling_of(typename KeyOf<DIM>::type a, typename KeyOf<DIM>::type b)
{
    int da, db;
    uint32_t ca[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
    unpack_key<DIM>(a, da, ca);
    unpack_key<DIM>(b, db, cb);
    if (da != db || da == 0) return false;
    for (int k = 0; k < DIM; k++)
        if ((ca[k] >> 1) != (cb[k] >> 1)) return false;
    return true;
}

template <int DIM>
__device__ __forceinline__ int child_index(typename KeyOf<DIM>::type a)
{
    int d;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<DIM>(a, d, c);
    int ci = 0;
    for (int k = 0; k < DIM; k++) ci |= (int)(c[k] & 1) << k;
    return ci;
}

// first child of a complete sibling group that may be coarsened
template <int DIM>
__device__ __forceinline__ void amr_coarsen_body(const int blk, int E, const typename KeyOf<DIM>::type *key, const double *eta,
                                                     double tau_coarsen, const uint8_t *refine, const uint32_t *face,
                                                     uint8_t *cflag)
{
    constexpr int NK = 1 << DIM;
    const int e = blk * 256 + threadIdx.x;
    if (e >= E) return;
    bool ok = (key[e] & 15) > 0 && child_index<DIM>(key[e]) == 0 && e + NK <= E;
    for (int j = 1; j < NK && ok; j++) ok = sibling_of<DIM>(key[e], key[e + j]) && child_index<DIM>(key[e + j]) == j;
    for (int j = 0; j < NK && ok; j++) ok = eta[e + j] <= tau_coarsen && !refine[e + j];
    for (int j = 0; j < NK && ok; j++) {
        int d;
        uint32_t c[3] = {0, 0, 0};
        unpack_key<DIM>(key[e + j], d, c);
        for (int k = 0; k < DIM && ok; k++)
            for (int s = 0; s < 2 && ok; s++) {
                if (((c[k] & 1) == 0) == (s == 1)) continue;  // this face looks at a sibling
                const uint32_t ent = face[(long long)(2 * k + s) * E + e + j];
                const uint32_t kind = ent >> 30;
                if (kind == kFiner) ok = false;
                else if (kind == kSame && refine[ent & kIdMask30]) ok = false;
            }
    }
    cflag[e] = ok ? 1 : 0;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_amr_coarsen(int E, const typename KeyOf<DIM>::type *key, const double *eta,
                                                     double tau_coarsen, const uint8_t *refine, const uint32_t *face,
                                                     uint8_t *cflag)
{
    amr_coarsen_body<DIM>(blockIdx.x, E, key, eta, tau_coarsen, refine, face, cflag);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct AmrCoarsenOp {
    int E;
    const typename KeyOf<DIM>::type *key;
    const double *eta;
    double tau_coarsen;
    const uint8_t *refine;
    const uint32_t *face;
    uint8_t *cflag;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        amr_coarsen_body<DIM>(blk, E, key, eta, tau_coarsen, refine, face, cflag);
    }
};


template <int DIM>
__device__ __forceinline__ void amr_emit_body(const int blk, int E, const typename KeyOf<DIM>::type *key, const uint8_t *refine,
                                                  const uint8_t *cflag, const int *cnt, const int *off,
                                                  const int *block_off, typename KeyOf<DIM>::type *key_new,
                                                  uint8_t *xkind, int32_t *xsrc, uint8_t *xchild)
{
    // off: exclusive scan of cnt within blocks of 1024 leaves; block_off:
    // exclusive scan of the blocks' totals
    const int e = blk * 256 + threadIdx.x;
    if (e >= E || cnt[e] == 0) return;
    int d;
    uint32_t c[3] = {0, 0, 0};
    unpack_key<DIM>(key[e], d, c);
    const int o = off[e] + block_off[e >> 10];
    if (refine[e]) {
        for (int ci = 0; ci < (1 << DIM); ci++) {
            uint32_t cc[3] = {0, 0, 0};
            for (int k = 0; k < DIM; k++) cc[k] = 2 * c[k] + ((ci >> k) & 1);
            key_new[o + ci] = pack_key<DIM>(d + 1, cc);
            xkind[o + ci] = 1;
            xsrc[o + ci] = e;
            xchild[o + ci] = (uint8_t)ci;
        }
    } else if (cflag[e]) {
        uint32_t cp[3] = {0, 0, 0};
        for (int k = 0; k < DIM; k++) cp[k] = c[k] >> 1;
        key_new[o] = pack_key<DIM>(d - 1, cp);
        xkind[o] = 2;
        xsrc[o] = e;
        xchild[o] = 0;
    } else {
        key_new[o] = key[e];
        xkind[o] = 0;
        xsrc[o] = e;
        xchild[o] = 0;
    }
}

template <int DIM>
__global__ __launch_bounds__(256) void k_amr_emit(int E, const typename KeyOf<DIM>::type *key, const uint8_t *refine,
                                                  const uint8_t *cflag, const int *cnt, const int *off,
                                                  const int *block_off, typename KeyOf<DIM>::type *key_new,
                                                  uint8_t *xkind, int32_t *xsrc, uint8_t *xchild)
{
    amr_emit_body<DIM>(blockIdx.x, E, key, refine, cflag, cnt, off, block_off, key_new, xkind, xsrc, xchild);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct AmrEmitOp {
    int E;
    const typename KeyOf<DIM>::type *key;
    const uint8_t *refine;
    const uint8_t *cflag;
    const int *cnt;
    const int *off;
    const int *block_off;
    typename KeyOf<DIM>::type *key_new;
    uint8_t *xkind;
    int32_t *xsrc;
    uint8_t *xchild;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        amr_emit_body<DIM>(blk, E, key, refine, cflag, cnt, off, block_off, key_new, xkind, xsrc, xchild);
    }
};

// ---- exclusive scan of int counts (1024 items per block) --------------------
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// in-block exclusive scan of 4 items per thread; returns the block total
__device__ __forceinline__ int block_excl_scan4(int *x4)
{
    __shared__ int wsum[4];
    const int t0 = x4[0], t1 = t0 + x4[1], t2 = t1 + x4[2], t3 = t2 + x4[3];
    const int incl = wave_incl_scan(t3);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int wbase = 0, total = 0;
    for (int w = 0; w < 4; w++) {
        if (w < wave) wbase += wsum[w];
        total += wsum[w];
    }
    const int excl = wbase + incl - t3;
    x4[0] = excl;
    x4[1] = excl + t0;
    x4[2] = excl + t1;
    x4[3] = excl + t2;
    __syncthreads();
    return total;
}

// Leaves after adaptation per current leaf (2^d for a refined leaf, 0 for
// the later children of a coarsened parent, 1 otherwise), with the
// refine/coarsen tallies, and their block-local exclusive scan, in one
// launch: each thread counts four consecutive leaves, then the block scans.
template <int DIM>
__device__ __forceinline__ void amr_count_scan_body(const int blk, int E, const typename KeyOf<DIM>::type *key,
                                                        const uint8_t *refine, const uint8_t *cflag, int *cnt,
                                                        int *off, int *block_sums, unsigned long long *tallies)
{
    int x[4];
    const long long base = (long long)blk * 1024 + threadIdx.x * 4;
    for (int q = 0; q < 4; q++) {
        const long long el = base + q;
        int n = 0;
        if (el < E) {
            const int e = (int)el;
            n = 1;
            if (refine[e]) {
                n = 1 << DIM;
                atomicAdd(&tallies[0], 1ull);
            } else if (cflag[e]) {
                atomicAdd(&tallies[1], 1ull);
            } else {
                const int ci = child_index<DIM>(key[e]);
                if (ci > 0 && e - ci >= 0 && cflag[e - ci] && sibling_of<DIM>(key[e - ci], key[e])) n = 0;
            }
            cnt[e] = n;
        }
        x[q] = n;
    }
    const int tot = block_excl_scan4(x);
    for (int q = 0; q < 4; q++)
        if (base + q < E) off[base + q] = x[q];
    if (threadIdx.x == 0) block_sums[blk] = tot;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_amr_count_scan(int E, const typename KeyOf<DIM>::type *key,
                                                        const uint8_t *refine, const uint8_t *cflag, int *cnt,
                                                        int *off, int *block_sums, unsigned long long *tallies)
{
    amr_count_scan_body<DIM>(blockIdx.x, E, key, refine, cflag, cnt, off, block_sums, tallies);
}

// its arguments, for a launch over many simulations (k_multi)
template <int DIM>
struct AmrCountScanOp {
    int E;
    const typename KeyOf<DIM>::type *key;
    const uint8_t *refine;
    const uint8_t *cflag;
    int *cnt;
    int *off;
    int *block_sums;
    unsigned long long *tallies;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        amr_count_scan_body<DIM>(blk, E, key, refine, cflag, cnt, off, block_sums, tallies);
    }
};

// one block scans the block sums in chunks of 1024; total to *total
__device__ __forceinline__ void scan_sums_body(const int blk, int nb, int *sums, int *total)
{
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        int x[4];
        const int base = c0 + threadIdx.x * 4;
        for (int q = 0; q < 4; q++) x[q] = base + q < nb ? sums[base + q] : 0;
        const int tot = block_excl_scan4(x);
        const int cbase = carry;
        for (int q = 0; q < 4; q++)
            if (base + q < nb) sums[base + q] = x[q] + cbase;
        __syncthreads();
        if (threadIdx.x == 0) carry = cbase + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void k_scan_sums(int nb, int *sums, int *total)
{
    scan_sums_body(blockIdx.x, nb, sums, total);
}

// its arguments, for a launch over many simulations (k_multi)
struct ScanSumsOp {
    int nb;
    int *sums;
    int *total;
    __device__ __forceinline__ void operator()(const int blk) const
    {
        scan_sums_body(blk, nb, sums, total);
    }
};

}  // namespace mdlts
