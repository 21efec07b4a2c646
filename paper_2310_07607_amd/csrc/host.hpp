// host.hpp -- host-side data structures of the library: 1-D reference
// tables of the Gauss-Legendre nodal DG basis, the linear forest (leaves in
// canonical order, hashed lookup, face tables) and the adaptation planner.
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace mdlts {

constexpr int kMaxM = 4;  // nodes per direction (order <= 3)

// Face neighbour kinds in the canonical face table (bits 30..31 of an entry).
enum FaceKind : uint32_t { kBoundary = 0, kSame = 1, kCoarser = 2, kFiner = 3 };

// 1-D tables of the degree-p Lagrange basis through the p+1 Gauss-Legendre
// nodes on [-1,1] (Sec. 2.1), all in FP64.
struct RefTables {
    int m = 0;
    double xi[kMaxM], w[kMaxM];
    double D1[kMaxM][kMaxM];      // D1[a][b] = l_b'(xi_a)
    double A[kMaxM][kMaxM];       // volume: (1/w_a) sum_q w_q D1[q][a] D1[q][b]
    double B[2][kMaxM];           // B[s][b] = l_b(-1 | +1)
    double G[2][kMaxM];           // G[s][b] = l_b'(-1 | +1)
    double Isub[2][kMaxM][kMaxM]; // Isub[pos][g][b] = l_b((xi_g + 2 pos - 1)/2)
    double Lsub[2][kMaxM][kMaxM]; // Lsub[pos][a][g] = w_g Isub[pos][g][a] / (2 w_a)
};
bool make_ref_tables(int p, RefTables &T);

// Gershgorin row-sum bound of the 1-D own block M^-1 K_ee of a unit element
// (h = 1, D = 1) with the given kinds on its lower/upper faces.  The d-D
// block of an axis-aligned box with diagonal D is the Kronecker sum of these
// (scaled by D_kk/h_k^2); its rows have negative diagonals, so the maximum
// row sum is the sum over directions of the 1-D maxima.
// Returns false if some diagonal entry is not negative (gamma too small).
bool gershgorin_table(const RefTables &T, double gamma, double out[4][4]);

// A diffusion tensor D (Sec. 2: D = kappa / (chi C_m)) as the library keeps
// it: diagonal and off-diagonal entries.  Accepted are symmetric positive
// definite tensors; in 2-D the z row and column must be zero.
struct Conductivity {
    double Dk[3] = {0, 0, 0};  // Dxx, Dyy, Dzz
    double Dx[3] = {0, 0, 0};  // Dxy, Dxz, Dyz
    bool full = false;         // some off-diagonal entry is nonzero
};
// D_sym = Dxx, Dyy, Dzz, Dxy, Dxz, Dyz; false if not accepted
bool parse_conductivity(const double D_sym[6], int dim, Conductivity &C);

// Gershgorin row-sum bound max_i sum_j |(M_e^-1 K_ee)_ij| of the own block of
// a root element (box h0) under a full tensor, for every combination of the
// kinds of its 2 dim faces: out[sum_f kind_f 4^f], face f = 2k + s.  The
// block of a leaf at depth d is 4^d times the root's.  Assembled from the
// tensor-product basis at the GL nodes; returns false if some block has a
// diagonal entry that is not negative (gamma too small).
bool own_block_table(const RefTables &T, int dim, const double h0[3], const Conductivity &C, double gamma,
                     std::vector<double> &out);

struct Leaf {
    uint8_t depth;
    uint32_t c[3];  // cell index in the level-`depth` grid of the whole box
};

struct Forest {
    int dim = 2, max_depth = 0;
    int n[3] = {1, 1, 1};
    std::vector<Leaf> leaves;             // canonical order
    std::vector<uint32_t> face;           // [2*dim][E]: kind<<30 | canonical id (or fine group)
    std::vector<uint32_t> fine;           // [groups][2^(dim-1)] canonical ids
    // lookup: the leaves of root r are [root_start[r], root_start[r+1]) and,
    // inside a root, sorted by the Morton key of their lower corner at the
    // depth cap (pre-order of a 2^d-tree with child bit k = dimension k)
    std::vector<int32_t> root_start;
    std::vector<uint32_t> mkey;

    int n_faces() const { return 2 * dim; }
    int n_sub() const { return 1 << (dim - 1); }
    size_t size() const { return leaves.size(); }

    void init_roots();
    // returns false for malformed, too deep, or unbalanced streams
    bool parse_bits(const uint8_t *bits, size_t n_bits);
    void write_bits(std::vector<uint8_t> &out) const;
    // lookup tables and face table; false if 2:1 balance is violated
    bool build_faces();
    // the leaf containing the lower corner of cell c at `depth`, or -1
    int64_t containing(int depth, const int64_t *c) const;
    uint32_t morton(int depth, const int64_t *local) const;
};

// Adaptation plan (Algorithm 1 thresholds; 2:1 closure; balanced coarsening).
// For each new leaf: kind (0 copy, 1 prolong from parent, 2 restrict from
// 2^d children), source old leaf (parent, or first child), child index.
struct AdaptPlan {
    Forest next;
    std::vector<uint8_t> kind;
    std::vector<int32_t> src;
    std::vector<uint8_t> child;
    int64_t n_refined = 0, n_coarsened = 0;
};
bool plan_adapt(const Forest &cur, const double *eta, double tau_refine, double tau_coarsen, AdaptPlan &plan);

// Per-leaf CFL with the separable Gershgorin bound (host reference of the
// device level kernel) and the resulting level.
void host_cfl(const Forest &F, const double h0[3], const double Dk[3], const double G[4][4], double *cfl);
// The same from the full-tensor table of own_block_table.
void host_cfl_full(const Forest &F, const std::vector<double> &table, double *cfl);
int level_of(double dt_barrier, double cfl);

}  // namespace mdlts
