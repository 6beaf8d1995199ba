// Internal structures of libseird (host and device views).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "seird.h"

namespace seird {

constexpr int NC = 5;

// Error plumbing: functions throw seird::Error, the C ABI converts it.
struct Error {
  int code;
  std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define HIPCHECK(x) ::seird::hip_check((x), #x)

// Where device memory comes from.  Without an active arena: hipMalloc.
// With one (set for the duration of a creation inside a caller's
// workspace): bump allocation of 256-byte aligned pieces of the workspace,
// SEIRD_ERR_WORKSPACE when it runs out.  A measuring arena allocates and
// copies nothing and only adds up the sizes (seird_workspace_bytes); code
// that touches device memory during a creation checks measuring() first.
struct Arena {
  uint8_t *base = nullptr;
  size_t cap = 0, used = 0;
  bool measure = false;
  void *take(size_t bytes);
};
Arena *&active_arena();  // thread-local; null = hipMalloc
bool measuring();
// makes `a` the active arena until the guard ends
struct ArenaScope {
  Arena *prev;
  explicit ArenaScope(Arena *a) : prev(active_arena()) { active_arena() = a; }
  ~ArenaScope() { active_arena() = prev; }
};
// device ranges owned by callers (their workspaces): dev_free skips them
void register_workspace(const void *base, size_t bytes);
void unregister_workspace(const void *base);

void *dev_alloc_bytes(size_t bytes);
template <class T>
T *dev_alloc(size_t n) {
  return static_cast<T *>(dev_alloc_bytes((n == 0 ? 1 : n) * sizeof(T)));
}
template <class T>
T *dev_upload(const std::vector<T> &v) {
  T *p = dev_alloc<T>(v.size());
  if (!v.empty() && !measuring()) HIPCHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}
void dev_free(void *p);

// ---------------------------------------------------------------------
// Mesh-level data built once per problem (Section 2.2).
//
// Node graph: for node i, its neighbours (sharing a triangle, itself
// excluded) sorted; a "slot" is a position in this CSR, i.e. one
// off-diagonal node block of the Jacobian.
//
// Incidence records (node-gather assembly): for every (triangle T, local
// vertex k), with i = T[k], j = T[k+1], l = T[k+2]:
//   Kii, Kij, Kil  (row i of the element stiffness K^T)
//   j, l and the slots of (i,j), (i,l) in row i.
// Grouped by i so that one thread assembles one node row without atomics.
// ---------------------------------------------------------------------
struct MeshHost {
  int64_t n = 0, nt = 0;
  std::vector<double> xy;       // node coordinates [n][2] (local orderings)
  std::vector<int64_t> rowptr;  // [n+1]
  std::vector<int32_t> col;     // [nslots]
  std::vector<int32_t> tslot;   // slot (i,j) -> slot (j,i)
  std::vector<double> mass;     // lumped mass [n]
  std::vector<int64_t> inc_ptr; // [n+1]
  std::vector<int32_t> inc_j, inc_l, inc_sj, inc_sl;
  std::vector<double> inc_K;    // [ninc][3]: Kii, Kij, Kil
  // per off-diagonal slot (i, j): its row i, and the (at most two)
  // incidence records of row i whose element holds edge (i, j), in record
  // order, as 2 k + w (w = 0: j is the record's first other vertex, 1:
  // its second), -1 when absent
  std::vector<int32_t> slot_row;
  std::vector<int32_t> slot_ek;  // [nslots][2]
  // assembled P1 stiffness: K_ii [n], K_ij [nslots], and per slot (i, j)
  // the sum of K^T_ii over the elements holding edge (i, j)
  std::vector<double> kd, ko, kw;
  // consistent mass M_ij = int phi_i phi_j: diagonal [n], slot values [nslots]
  std::vector<double> cmass_d, cmass_o;
  // boundary edges (in exactly one triangle), per node: the other end and
  // the outward normal scaled by the edge length
  std::vector<int64_t> bnd_ptr;  // [n+1]
  std::vector<int32_t> bnd_j;
  std::vector<double> bnd_nl;    // [nb][2]
};

struct MeshDev {
  int64_t n = 0, nslots = 0;
  int64_t *rowptr = nullptr;
  int32_t *col = nullptr;
  int32_t *tslot = nullptr;
  double *mass = nullptr;
  int64_t *inc_ptr = nullptr;
  int32_t *inc_j = nullptr, *inc_l = nullptr, *inc_sj = nullptr, *inc_sl = nullptr;
  double *inc_K = nullptr;
  int32_t *slot_row = nullptr, *slot_ek = nullptr;
  double *kd = nullptr, *ko = nullptr, *kw = nullptr;
  // discretisation variants: consistent mass (null: lumped) and boundary
  // flux data [n][5][2] (null: homogeneous Neumann)
  const double *cmass_d = nullptr, *cmass_o = nullptr;
  const int64_t *bnd_ptr = nullptr;
  const int32_t *bnd_j = nullptr;
  const double *bnd_nl = nullptr;
  const double *qflux = nullptr;
  // batches: instance of every node and the parameters of every instance
  // (both null for a single problem)
  const int32_t *inst = nullptr;
  const struct ParamsDev *Pinst = nullptr;
};

struct ParamsDev {
  double sigma, gE, gR, gD, A, alpha, mu, bI, bE;
  double nu[5];
};

// ---------------------------------------------------------------------
// Subdomain matrices: local unknowns l = 5*p + c for local node p (local
// ordering by reverse Cuthill-McKee or a strip sort, whichever has the
// smaller bandwidth).  After factorisation the diagonal tile of a row holds
// the strictly-lower part of L_KK^{-1} and the upper part of U_KK^{-1}; the
// other tiles hold L (left of the diagonal) and U (right of it).  Padded
// rows (n_loc .. nt*t - 1) carry an identity diagonal.
// ---------------------------------------------------------------------
// Factor storage of one system in 32x32 (or 16x16) row-major tiles.
// Envelope layout (env_off >= 0, the subdomains): tile row K holds tile
// columns lo_K .. hi_K contiguously, from tile offset row_K; lo is
// nondecreasing and the envelope is symmetric (tile (K, J), J > K, is
// stored iff lo_J <= K), so LU without pivoting keeps its fill inside it.
// row_K and lo_K are in the row table at env_off + K (nt + 1 entries).
// Band layout (env_off < 0, the coarse system): row K holds tile columns
// K - bl .. K + bu at slots 0 .. bl + bu.
struct SubInfo {
  int64_t base;     // offset (entries) of the factor storage
  int32_t n_loc;    // local unknowns (5 * local nodes)
  int32_t nt;       // number of tile rows
  int32_t bl, bu;   // block bandwidths (largest extent left / right of the diagonal)
  int32_t l2g_off;  // offset into the local->global unknown map
  int32_t env_off;  // offset into the row table, or -1 for the band layout
};

struct ExtractEntry {  // one node block of R_i A R_i^T
  int32_t sub;
  int32_t p, q;        // local node positions (row block, column block)
  int32_t ref;         // >= 0: off-diagonal slot; < 0: diagonal of node -ref-1
};

struct PrecondHost {
  int n_sub = 0, overlap = 0, tile = 32, prec = 0;
  int bs = NC;                        // unknowns per node: 5 (coupled) or 1 (one compartment)
  std::vector<SubInfo> subs;          // subdomains (then, if two-level, coarse)
  std::vector<int32_t> l2g;           // local unknown -> global unknown
  std::vector<uint8_t> owned;         // per local unknown: owned by the sub
  std::vector<ExtractEntry> extract;  // block entries, grouped by (subdomain, local node)
  std::vector<int32_t> ent_ptr;       // first entry of each local node (all subdomains in order) [+1]
  std::vector<int32_t> trow_ptr;      // first tile row of each subdomain in a global count [n_sub+1]
  std::vector<int32_t> trow_sub;      // subdomain of each such tile row
  int32_t max_node_blocks = 0;        // most extraction entries of one local node
  std::vector<int32_t> order;         // subdomain processing order (LPT)
  std::vector<int32_t> env_row, env_lo;  // subdomain row tables (tile offset, first tile column)
  int64_t factor_entries = 0;   // subdomain tile-envelope entries
  // flops of the subdomain factorisation over the tile envelopes: tile
  // products as the matrix cores execute them (dense 2 T^3 per product:
  // the U and L panel tiles and every Schur update), and the useful count
  // (triangular-times-dense panel products at T^3) plus the diagonal tiles'
  // LU and two triangular inverses (4/3 T^3 each, vector ALUs)
  double lu_mfma_flops = 0.0, lu_useful_flops = 0.0;
  int64_t coarse_entries = 0;   // coarse band entries (own buffer)
  int32_t max_nodes = 0, max_bw = 0;
  int32_t max_nloc = 0;
  double mean_bw = 0.0;
  int32_t coarse_bw = 0;
  // two-level
  bool two_level = false;
  int64_t nc = 0;                      // coarse nodes
  std::vector<int64_t> z_ptr;          // Z rows (fine nodes) [n+1]
  std::vector<int32_t> z_col;
  std::vector<double> z_val;
  std::vector<int64_t> zt_ptr;         // Z^T rows (coarse nodes) [nc+1]
  std::vector<int32_t> zt_col;
  std::vector<double> zt_val;
  SubInfo coarse;                      // coarse tile-band geometry
  std::vector<int32_t> c_perm;         // coarse node -> coarse local position
  // Galerkin map: coarse block k (position pair) gets sum w * fine block
  std::vector<int32_t> gal_p, gal_q;   // coarse local positions of block k
  std::vector<int64_t> gal_ptr;        // [nblocks+1]
  std::vector<int32_t> gal_ref;        // fine block ref (as ExtractEntry.ref)
  std::vector<double> gal_w;
  // the coarse system as a graph over coarse positions, for the Krylov
  // coarse solver (two-grid RAS-V2): adjacency without self loops, node
  // points, the fine subdomain that owns each coarse node's own fine node,
  // and where Galerkin block k goes (-p-1: diagonal block of position p;
  // >= 0: slot of the coarse graph)
  std::vector<int64_t> cg_rowptr;
  std::vector<int32_t> cg_col;
  std::vector<double> cg_xy;
  std::vector<int32_t> cg_owner;
  std::vector<int32_t> gal_dst;
};

void build_mesh(int64_t n, const double *xy, int64_t nt, const int32_t *tri,
                MeshHost &m);
void build_precond(const MeshHost &m, const seird_schwarz_opts &o, const int32_t *part,
                   PrecondHost &ph, int bs = NC);

}  // namespace seird
