// host.cpp -- reference tables, linear forest and adaptation planner.
// Compiled with -ffp-contract=off: the CFL arithmetic here is the host
// reference of the device level kernel and must round the same way.
#include "host.hpp"

#include <cmath>
#include <cstring>

namespace mdlts {

// ---------------------------------------------------------------------------
// 1-D reference tables (Sec. 2.1: Lagrange basis at the Gauss-Legendre nodes)
// ---------------------------------------------------------------------------
static double lagrange_value(const RefTables &T, const double *lam, int b, double x)
{
    // l_b(x) = lambda_b * prod_{k != b} (x - xi_k), lambda_b the barycentric weight
    double v = lam[b];
    for (int k = 0; k < T.m; k++)
        if (k != b) v *= (x - T.xi[k]);
    return v;
}

static double lagrange_deriv(const RefTables &T, const double *lam, int b, double x)
{
    // d/dx of the product: sum over the factor that is differentiated
    double s = 0.0;
    for (int k = 0; k < T.m; k++) {
        if (k == b) continue;
        double v = lam[b];
        for (int q = 0; q < T.m; q++)
            if (q != b && q != k) v *= (x - T.xi[q]);
        s += v;
    }
    return s;
}

bool make_ref_tables(int p, RefTables &T)
{
    T = RefTables{};
    if (p == 1) {
        T.m = 2;
        const double r = 1.0 / std::sqrt(3.0);
        T.xi[0] = -r; T.xi[1] = r;
        T.w[0] = 1.0; T.w[1] = 1.0;
    } else if (p == 2) {
        T.m = 3;
        const double r = std::sqrt(0.6);
        T.xi[0] = -r; T.xi[1] = 0.0; T.xi[2] = r;
        T.w[0] = 5.0 / 9.0; T.w[1] = 8.0 / 9.0; T.w[2] = 5.0 / 9.0;
    } else if (p == 3) {
        // roots of P_4: x^2 = 3/7 -+ (2/7) sqrt(6/5); weights (18 +- sqrt(30))/36
        T.m = 4;
        const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2));
        const double b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
        T.xi[0] = -b; T.xi[1] = -a; T.xi[2] = a; T.xi[3] = b;
        const double wa = (18.0 + std::sqrt(30.0)) / 36.0, wb = (18.0 - std::sqrt(30.0)) / 36.0;
        T.w[0] = wb; T.w[1] = wa; T.w[2] = wa; T.w[3] = wb;
    } else {
        return false;
    }
    const int m = T.m;
    double lam[kMaxM];
    for (int j = 0; j < m; j++) {
        double d = 1.0;
        for (int k = 0; k < m; k++)
            if (k != j) d *= (T.xi[j] - T.xi[k]);
        lam[j] = 1.0 / d;
    }
    for (int a = 0; a < m; a++) {
        double diag = 0.0;
        for (int b = 0; b < m; b++) {
            if (a == b) continue;
            T.D1[a][b] = (lam[b] / lam[a]) / (T.xi[a] - T.xi[b]);
            diag -= T.D1[a][b];
        }
        T.D1[a][a] = diag;  // rows of a differentiation matrix sum to zero
    }
    for (int a = 0; a < m; a++)
        for (int b = 0; b < m; b++) {
            double s = 0.0;
            for (int q = 0; q < m; q++) s += T.w[q] * T.D1[q][a] * T.D1[q][b];
            T.A[a][b] = s / T.w[a];
        }
    for (int s = 0; s < 2; s++) {
        const double x = s ? 1.0 : -1.0;
        for (int b = 0; b < m; b++) {
            T.B[s][b] = lagrange_value(T, lam, b, x);
            T.G[s][b] = lagrange_deriv(T, lam, b, x);
        }
    }
    for (int pos = 0; pos < 2; pos++)
        for (int g = 0; g < m; g++)
            for (int b = 0; b < m; b++)
                T.Isub[pos][g][b] = lagrange_value(T, lam, b, 0.5 * (T.xi[g] + 2.0 * pos - 1.0));
    for (int pos = 0; pos < 2; pos++)
        for (int a = 0; a < m; a++)
            for (int g = 0; g < m; g++) T.Lsub[pos][a][g] = T.w[g] * T.Isub[pos][g][a] / (2.0 * T.w[a]);
    return true;
}

bool gershgorin_table(const RefTables &T, double gamma, double out[4][4])
{
    const int m = T.m;
    // penalty factor 1/2 (1 + h/h_nbr) per kind; boundary faces carry no terms
    const double factor[4] = {0.0, 1.0, 0.75, 1.5};
    for (int lo = 0; lo < 4; lo++)
        for (int hi = 0; hi < 4; hi++) {
            double K[kMaxM][kMaxM];
            for (int i = 0; i < m; i++)
                for (int j = 0; j < m; j++) {
                    // unit element [0,1]: dx = dxi/2, d/dx = 2 d/dxi, weights w/2
                    double s = 0.0;
                    for (int q = 0; q < m; q++) s += T.w[q] * T.D1[q][i] * T.D1[q][j];
                    K[i][j] = -2.0 * s;
                }
            const int kinds[2] = {lo, hi};
            for (int side = 0; side < 2; side++) {
                if (kinds[side] == kBoundary) continue;
                const double nrm = side ? 1.0 : -1.0;
                const double sigma = gamma * factor[kinds[side]];
                for (int i = 0; i < m; i++)
                    for (int j = 0; j < m; j++) {
                        const double dj = nrm * 2.0 * T.G[side][j], di = nrm * 2.0 * T.G[side][i];
                        K[i][j] += 0.5 * dj * T.B[side][i] + 0.5 * T.B[side][j] * di -
                                   sigma * T.B[side][j] * T.B[side][i];
                    }
            }
            double worst = 0.0;
            for (int i = 0; i < m; i++) {
                const double Mi = 0.5 * T.w[i];
                if (!(K[i][i] < 0.0)) return false;
                double r = 0.0;
                for (int j = 0; j < m; j++) r += std::fabs(K[i][j] / Mi);
                if (r > worst) worst = r;
            }
            out[lo][hi] = worst;
        }
    return true;
}

bool parse_conductivity(const double D_sym[6], int dim, Conductivity &C)
{
    if (!D_sym) return false;
    for (int q = 0; q < 6; q++)
        if (!std::isfinite(D_sym[q])) return false;
    C = Conductivity{};
    for (int k = 0; k < 3; k++) C.Dk[k] = D_sym[k];
    for (int q = 0; q < 3; q++) C.Dx[q] = D_sym[3 + q];
    if (dim == 2 && (C.Dx[1] != 0.0 || C.Dx[2] != 0.0)) return false;
    // positive definite: positive leading principal minors of the dim x dim tensor
    const double a = C.Dk[0], b = C.Dk[1], c = C.Dk[2], xy = C.Dx[0], xz = C.Dx[1], yz = C.Dx[2];
    for (int k = 0; k < dim; k++)
        if (!(C.Dk[k] > 0.0)) return false;
    if (!(a * b - xy * xy > 0.0)) return false;
    if (dim == 3 && !(a * (b * c - yz * yz) - xy * (xy * c - yz * xz) + xz * (xy * yz - b * xz) > 0.0)) return false;
    C.full = xy != 0.0 || xz != 0.0 || yz != 0.0;
    return true;
}

bool own_block_table(const RefTables &T, int dim, const double h0[3], const Conductivity &C, double gamma,
                     std::vector<double> &out)
{
    const int m = T.m;
    const int np = dim == 2 ? m * m : m * m * m;
    const int nfaces = 2 * dim;
    const double D[3][3] = {{C.Dk[0], C.Dx[0], C.Dx[1]}, {C.Dx[0], C.Dk[1], C.Dx[2]}, {C.Dx[1], C.Dx[2], C.Dk[2]}};
    auto digit = [&](int i, int k) {
        for (int q = 0; q < k; q++) i /= m;
        return i % m;
    };
    std::vector<double> Mi(np);
    for (int i = 0; i < np; i++) {
        double v = 1.0;
        for (int k = 0; k < dim; k++) v *= T.w[digit(i, k)] * 0.5 * h0[k];
        Mi[i] = v;
    }
    // value and physical gradient of basis function j at a point given by
    // the 1-D basis values val1[k][b] and derivatives der1[k][b] there
    // (tensor products of the 1-D factors)
    auto grad_at = [&](int j, const double *val1, const double *der1, double *g, double &val) {
        val = 1.0;
        for (int k = 0; k < dim; k++) val *= val1[k * kMaxM + digit(j, k)];
        for (int l = 0; l < dim; l++) {
            double v = 2.0 / h0[l] * der1[l * kMaxM + digit(j, l)];
            for (int k = 0; k < dim; k++)
                if (k != l) v *= val1[k * kMaxM + digit(j, k)];
            g[l] = v;
        }
    };
    // volume: -int D grad(l_j) . grad(l_i), GL rule at the nodes
    std::vector<double> V((size_t)np * np, 0.0);
    std::vector<double> gq((size_t)np * 3), vq(np);
    for (int q = 0; q < np; q++) {
        int qi[3] = {0, 0, 0};
        double val1[3 * kMaxM] = {}, der1[3 * kMaxM] = {};
        double Wq = 1.0;
        for (int k = 0; k < dim; k++) {
            qi[k] = digit(q, k);
            Wq *= T.w[qi[k]] * 0.5 * h0[k];
            for (int b = 0; b < m; b++) {
                val1[k * kMaxM + b] = b == qi[k] ? 1.0 : 0.0;
                der1[k * kMaxM + b] = T.D1[qi[k]][b];
            }
        }
        for (int j = 0; j < np; j++) grad_at(j, val1, der1, &gq[(size_t)j * 3], vq[j]);
        for (int i = 0; i < np; i++)
            for (int j = 0; j < np; j++) {
                double a = 0.0;
                for (int x = 0; x < dim; x++)
                    for (int y = 0; y < dim; y++) a += gq[(size_t)i * 3 + x] * D[x][y] * gq[(size_t)j * 3 + y];
                V[(size_t)i * np + j] -= Wq * a / Mi[i];
            }
    }
    // own-side terms of face f with the neighbour frozen at zero:
    // consistency and symmetry (Cf) and the penalty without sigma (Pf)
    std::vector<double> Cf((size_t)nfaces * np * np, 0.0), Pf((size_t)nfaces * np * np, 0.0);
    const int nf = np / m;
    for (int f = 0; f < nfaces; f++) {
        const int k = f / 2, s = f % 2;
        const double ns = s ? 1.0 : -1.0;
        for (int g = 0; g < nf; g++) {
            int qi[3] = {0, 0, 0};
            double val1[3 * kMaxM] = {}, der1[3 * kMaxM] = {};
            double Wg = 1.0;
            int gg = g;
            for (int t = 0; t < dim; t++) {
                if (t == k) {
                    for (int b = 0; b < m; b++) {
                        val1[t * kMaxM + b] = T.B[s][b];
                        der1[t * kMaxM + b] = T.G[s][b];
                    }
                    continue;
                }
                qi[t] = gg % m;
                gg /= m;
                Wg *= T.w[qi[t]] * 0.5 * h0[t];
                for (int b = 0; b < m; b++) {
                    val1[t * kMaxM + b] = b == qi[t] ? 1.0 : 0.0;
                    der1[t * kMaxM + b] = T.D1[qi[t]][b];
                }
            }
            for (int j = 0; j < np; j++) grad_at(j, val1, der1, &gq[(size_t)j * 3], vq[j]);
            for (int i = 0; i < np; i++) {
                double dni = 0.0;
                for (int y = 0; y < dim; y++) dni += D[k][y] * gq[(size_t)i * 3 + y];
                dni *= ns;
                for (int j = 0; j < np; j++) {
                    double dnj = 0.0;
                    for (int y = 0; y < dim; y++) dnj += D[k][y] * gq[(size_t)j * 3 + y];
                    dnj *= ns;
                    const size_t o = ((size_t)f * np + i) * np + j;
                    Cf[o] += Wg * (0.5 * dnj * vq[i] + 0.5 * vq[j] * dni) / Mi[i];
                    Pf[o] += Wg * vq[j] * vq[i] / Mi[i];
                }
            }
        }
    }
    // penalty sigma = gamma 1/2 (D_kk/h + D_kk/h_nbr) per kind
    const double factor[4] = {0.0, 1.0, 0.75, 1.5};
    const int n_combo = 1 << (2 * nfaces);
    out.assign((size_t)n_combo, 0.0);
    std::vector<double> L((size_t)np * np);
    for (int combo = 0; combo < n_combo; combo++) {
        L = V;
        for (int f = 0; f < nfaces; f++) {
            const int kind = (combo >> (2 * f)) & 3;
            if (kind == kBoundary) continue;
            const int k = f / 2;
            const double sigma = gamma * D[k][k] / h0[k] * factor[kind];
            const double *cf = &Cf[(size_t)f * np * np], *pf = &Pf[(size_t)f * np * np];
            for (size_t o = 0; o < (size_t)np * np; o++) L[o] += cf[o] - sigma * pf[o];
        }
        double worst = 0.0;
        for (int i = 0; i < np; i++) {
            if (!(L[(size_t)i * np + i] < 0.0)) return false;
            double r = 0.0;
            for (int j = 0; j < np; j++) r += std::fabs(L[(size_t)i * np + j]);
            if (r > worst) worst = r;
        }
        out[(size_t)combo] = worst;
    }
    return true;
}

// ---------------------------------------------------------------------------
// linear forest
// ---------------------------------------------------------------------------
void Forest::init_roots()
{
    leaves.clear();
    leaves.reserve((size_t)n[0] * n[1] * n[2]);
    for (int z = 0; z < n[2]; z++)
        for (int y = 0; y < n[1]; y++)
            for (int x = 0; x < n[0]; x++) {
                Leaf L;
                L.depth = 0;
                L.c[0] = x; L.c[1] = y; L.c[2] = z;
                leaves.push_back(L);
            }
}

static bool parse_rec(Forest &F, int depth, const int64_t *c, const uint8_t *bits, size_t n_bits, size_t &pos)
{
    if (pos >= n_bits) return false;
    const uint8_t b = bits[pos++];
    if (b > 1) return false;
    if (b == 0) {
        Leaf L;
        L.depth = (uint8_t)depth;
        for (int k = 0; k < 3; k++) L.c[k] = (uint32_t)c[k];
        F.leaves.push_back(L);
        return true;
    }
    if (depth >= F.max_depth) return false;
    for (int ci = 0; ci < (1 << F.dim); ci++) {
        int64_t cc[3] = {0, 0, 0};
        for (int k = 0; k < F.dim; k++) cc[k] = 2 * c[k] + ((ci >> k) & 1);
        if (!parse_rec(F, depth + 1, cc, bits, n_bits, pos)) return false;
    }
    return true;
}

bool Forest::parse_bits(const uint8_t *bits, size_t n_bits)
{
    leaves.clear();
    leaves.reserve(n_bits);
    size_t pos = 0;
    for (int z = 0; z < n[2]; z++)
        for (int y = 0; y < n[1]; y++)
            for (int x = 0; x < n[0]; x++) {
                int64_t c[3] = {x, y, z};
                if (!parse_rec(*this, 0, c, bits, n_bits, pos)) return false;
            }
    if (pos != n_bits) return false;
    return build_faces();
}

static void write_rec(const Forest &F, int depth, const int64_t *c, size_t &pos, std::vector<uint8_t> &out)
{
    const Leaf &L = F.leaves[pos];
    bool same = L.depth == depth;
    for (int k = 0; k < F.dim && same; k++) same = (int64_t)L.c[k] == c[k];
    if (same) {
        out.push_back(0);
        pos++;
        return;
    }
    out.push_back(1);
    for (int ci = 0; ci < (1 << F.dim); ci++) {
        int64_t cc[3] = {0, 0, 0};
        for (int k = 0; k < F.dim; k++) cc[k] = 2 * c[k] + ((ci >> k) & 1);
        write_rec(F, depth + 1, cc, pos, out);
    }
}

void Forest::write_bits(std::vector<uint8_t> &out) const
{
    out.clear();
    out.reserve(leaves.size() * 2);
    size_t pos = 0;
    for (int z = 0; z < n[2]; z++)
        for (int y = 0; y < n[1]; y++)
            for (int x = 0; x < n[0]; x++) {
                int64_t c[3] = {x, y, z};
                write_rec(*this, 0, c, pos, out);
            }
}

static inline uint32_t spread2(uint32_t x)  // 8 bits -> even bits of 16
{
    x = (x | (x << 4)) & 0x0F0Fu;
    x = (x | (x << 2)) & 0x3333u;
    x = (x | (x << 1)) & 0x5555u;
    return x;
}

static inline uint32_t spread3(uint32_t x)  // 8 bits -> every third bit of 24
{
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

uint32_t Forest::morton(int depth, const int64_t *local) const
{
    // interleave the bits of the cell's corner at the depth cap, x lowest
    const int sh = max_depth - depth;
    if (dim == 2) return spread2((uint32_t)(local[0] << sh)) | (spread2((uint32_t)(local[1] << sh)) << 1);
    return spread3((uint32_t)(local[0] << sh)) | (spread3((uint32_t)(local[1] << sh)) << 1) |
           (spread3((uint32_t)(local[2] << sh)) << 2);
}

int64_t Forest::containing(int depth, const int64_t *c) const
{
    int64_t rc[3] = {0, 0, 0}, loc[3] = {0, 0, 0};
    for (int k = 0; k < dim; k++) {
        rc[k] = c[k] >> depth;
        loc[k] = c[k] - (rc[k] << depth);
    }
    const int64_t rid = rc[0] + (int64_t)n[0] * (rc[1] + (int64_t)n[1] * rc[2]);
    const uint32_t m = morton(depth, loc);
    // last leaf of the root whose key is <= m (the first key of a root is 0)
    const int64_t lo = root_start[rid];
    int64_t len = root_start[rid + 1] - lo;
    if (len <= 0) return -1;
    const uint32_t *base = &mkey[lo];
    while (len > 1) {
        const int64_t half = len >> 1;
        base = base[half] <= m ? base + half : base;
        len -= half;
    }
    return base - mkey.data();
}

bool Forest::build_faces()
{
    const size_t E = leaves.size();
    const size_t n_roots = (size_t)n[0] * n[1] * n[2];
    root_start.assign(n_roots + 1, 0);
    mkey.resize(E);
    {
        size_t e = 0;
        for (size_t r = 0; r < n_roots; r++) {
            root_start[r] = (int32_t)e;
            const int64_t rc[3] = {(int64_t)(r % n[0]), (int64_t)((r / n[0]) % n[1]),
                                   (int64_t)(r / ((size_t)n[0] * n[1]))};
            while (e < E) {
                const Leaf &L = leaves[e];
                bool in = true;
                int64_t loc[3] = {0, 0, 0};
                for (int k = 0; k < dim; k++) {
                    if (((int64_t)L.c[k] >> L.depth) != rc[k]) in = false;
                    loc[k] = (int64_t)L.c[k] - (rc[k] << L.depth);
                }
                if (!in) break;
                mkey[e] = morton(L.depth, loc);
                e++;
            }
        }
        root_start[n_roots] = (int32_t)e;
        if (e != E) return false;  // leaves not grouped by root in root order
    }
    face.assign((size_t)n_faces() * E, 0);
    fine.clear();
    for (size_t e = 0; e < E; e++) {
        const Leaf &L = leaves[e];
        for (int k = 0; k < dim; k++)
            for (int s = 0; s < 2; s++) {
                int64_t t[3] = {L.c[0], L.c[1], L.c[2]};
                t[k] += s ? 1 : -1;
                uint32_t entry = kBoundary << 30;
                if (t[k] >= 0 && t[k] < ((int64_t)n[k] << L.depth)) {
                    const int64_t id = containing(L.depth, t);
                    if (id < 0) return false;
                    const Leaf &N = leaves[id];
                    if (N.depth == L.depth) {
                        entry = (kSame << 30) | (uint32_t)id;
                    } else if (N.depth + 1 == L.depth) {
                        entry = (kCoarser << 30) | (uint32_t)id;
                    } else if (N.depth > L.depth) {
                        // the neighbour cell is refined: its children on
                        // this face must be leaves (2:1 balance)
                        const uint32_t g = (uint32_t)(fine.size() / n_sub());
                        const int want = s ? 0 : 1;
                        for (int ci = 0; ci < (1 << dim); ci++) {
                            if (((ci >> k) & 1) != want) continue;
                            int64_t cc[3] = {0, 0, 0};
                            for (int q = 0; q < dim; q++) cc[q] = 2 * t[q] + ((ci >> q) & 1);
                            const int64_t fid = containing(L.depth + 1, cc);
                            if (fid < 0 || leaves[fid].depth != L.depth + 1) return false;
                            fine.push_back((uint32_t)fid);
                        }
                        entry = (kFiner << 30) | g;
                    } else {
                        return false;  // coarser by more than one depth
                    }
                }
                face[(size_t)(2 * k + s) * E + e] = entry;
            }
    }
    return true;
}

// ---------------------------------------------------------------------------
// adaptation planner (Algorithm 1: refine eta >= tau_refine, coarsen
// eta <= tau_coarsen; 2:1 closure by refining coarser neighbours)
// ---------------------------------------------------------------------------
bool plan_adapt(const Forest &cur, const double *eta, double tau_refine, double tau_coarsen, AdaptPlan &plan)
{
    const size_t E = cur.size();
    const int nk = 1 << cur.dim;
    std::vector<uint8_t> refine(E, 0);
    std::vector<int32_t> work;
    for (size_t e = 0; e < E; e++)
        if (eta[e] >= tau_refine && cur.leaves[e].depth < cur.max_depth) {
            refine[e] = 1;
            work.push_back((int32_t)e);
        }
    while (!work.empty()) {
        const int32_t e = work.back();
        work.pop_back();
        for (int f = 0; f < cur.n_faces(); f++) {
            const uint32_t ent = cur.face[(size_t)f * E + e];
            if ((ent >> 30) != kCoarser) continue;
            const uint32_t nb = ent & 0x3fffffffu;
            if (!refine[nb]) {
                refine[nb] = 1;
                work.push_back((int32_t)nb);
            }
        }
    }
    // coarsening groups: 2^d consecutive sibling leaves
    std::vector<uint8_t> coarsen_first(E, 0);
    for (size_t e = 0; e + nk <= E; e++) {
        const Leaf &L = cur.leaves[e];
        if (L.depth == 0) continue;
        bool first = true;
        for (int k = 0; k < cur.dim; k++) first = first && (L.c[k] & 1) == 0;
        if (!first) continue;
        bool ok = true;
        for (int j = 0; j < nk && ok; j++) {
            const Leaf &C = cur.leaves[e + j];
            if (C.depth != L.depth) { ok = false; break; }
            for (int k = 0; k < cur.dim; k++)
                if (C.c[k] != L.c[k] + ((j >> k) & 1)) ok = false;
            if (!ok) break;
            if (!(eta[e + j] <= tau_coarsen) || refine[e + j]) ok = false;
        }
        for (int j = 0; j < nk && ok; j++) {
            const size_t ce = e + j;
            const Leaf &C = cur.leaves[ce];
            for (int k = 0; k < cur.dim && ok; k++)
                for (int s = 0; s < 2 && ok; s++) {
                    const int64_t t = (int64_t)C.c[k] + (s ? 1 : -1);
                    if ((t >> 1) == (int64_t)(C.c[k] >> 1)) continue;  // sibling
                    const uint32_t ent = cur.face[(size_t)(2 * k + s) * E + ce];
                    const uint32_t kind = ent >> 30;
                    if (kind == kFiner) ok = false;
                    else if (kind == kSame && refine[ent & 0x3fffffffu]) ok = false;
                }
        }
        if (ok) coarsen_first[e] = 1;
    }
    plan.next.dim = cur.dim;
    plan.next.max_depth = cur.max_depth;
    for (int k = 0; k < 3; k++) plan.next.n[k] = cur.n[k];
    plan.next.leaves.clear();
    plan.next.leaves.reserve(E + E / 2);
    plan.kind.clear();
    plan.src.clear();
    plan.child.clear();
    plan.n_refined = plan.n_coarsened = 0;
    for (size_t e = 0; e < E;) {
        const Leaf &L = cur.leaves[e];
        if (refine[e]) {
            for (int ci = 0; ci < nk; ci++) {
                Leaf C;
                C.depth = (uint8_t)(L.depth + 1);
                for (int k = 0; k < 3; k++) C.c[k] = k < cur.dim ? 2 * L.c[k] + ((ci >> k) & 1) : 0;
                plan.next.leaves.push_back(C);
                plan.kind.push_back(1);
                plan.src.push_back((int32_t)e);
                plan.child.push_back((uint8_t)ci);
            }
            plan.n_refined++;
            e++;
        } else if (coarsen_first[e]) {
            Leaf P;
            P.depth = (uint8_t)(L.depth - 1);
            for (int k = 0; k < 3; k++) P.c[k] = L.c[k] >> 1;
            plan.next.leaves.push_back(P);
            plan.kind.push_back(2);
            plan.src.push_back((int32_t)e);
            plan.child.push_back(0);
            plan.n_coarsened++;
            e += nk;
        } else {
            plan.next.leaves.push_back(L);
            plan.kind.push_back(0);
            plan.src.push_back((int32_t)e);
            plan.child.push_back(0);
            e++;
        }
    }
    return plan.next.build_faces();
}

void host_cfl(const Forest &F, const double h0[3], const double Dk[3], const double G[4][4], double *cfl)
{
    const size_t E = F.size();
    for (size_t e = 0; e < E; e++) {
        double s = 0.0;
        for (int k = 0; k < F.dim; k++) {
            const double h = std::ldexp(h0[k], -(int)F.leaves[e].depth);
            const uint32_t lo = F.face[(size_t)(2 * k) * E + e] >> 30;
            const uint32_t hi = F.face[(size_t)(2 * k + 1) * E + e] >> 30;
            s += Dk[k] / (h * h) * G[lo][hi];
        }
        cfl[e] = 1.0 / s;
    }
}

void host_cfl_full(const Forest &F, const std::vector<double> &table, double *cfl)
{
    const size_t E = F.size();
    for (size_t e = 0; e < E; e++) {
        uint32_t idx = 0;
        for (int f = 0; f < 2 * F.dim; f++) idx |= (F.face[(size_t)f * E + e] >> 30) << (2 * f);
        cfl[e] = 1.0 / (table[idx] * std::ldexp(1.0, 2 * (int)F.leaves[e].depth));
    }
}

int level_of(double dt_barrier, double cfl)
{
    int b = 0;
    while (b < 64 && std::ldexp(dt_barrier, -b) > cfl) b++;
    return b;
}

}  // namespace mdlts
