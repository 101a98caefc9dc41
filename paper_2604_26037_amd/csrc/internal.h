// Internal declarations of libpawfe (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "pawfe.h"

namespace pawfe {

constexpr int kNpMax = 7;    // degree <= 6
constexpr int kNqMax = 8;    // Gauss points per direction
constexpr int kNpjMax = 32;  // projectors per atom
constexpr int kMaxConcBlocks = 4;   // column blocks of a filter in flight at once

// Error helper: records the message for pawfe_last_error and returns the code.
pawfe_status fail(pawfe_status code, const std::string& msg);

#define PAWFE_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::pawfe::fail(PAWFE_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// 1-D reference tables handed to the cell kernels by value.
//   B[q*np + a] = l_a(eta_q), Lagrange basis through the GLL nodes at Gauss point q
//   K1[a*np + b] = sum_q w_q l_a'(eta_q) l_b'(eta_q)   (reference [-1,1])
//   M1[a*np + b] = sum_q w_q l_a(eta_q) l_b(eta_q)
//   f[d] = 1/2 det J (2/h_d)^2 (kinetic factor), detJ = hx hy hz / 8
template <typename T>
struct Tab1D {
  T B[kNqMax * kNpMax];
  T K1[kNpMax * kNpMax];
  T M1[kNpMax * kNpMax];
  T G1[kNpMax * kNpMax];   // G1[a][b] = sum_q w_q N_a N_b' (reference element)
  T f[3];
  T detJ;
  T g[3];                  // complex operators: -k_d det J (2/h_d) (imaginary local term)
  T w[kNqMax];             // 1-D Gauss weights (W_q = w_qx w_qy w_qz detJ), zero past nq
};

// Device-resident tables of one operator.
struct DeviceTables {
  Tab1D<double>* tab64 = nullptr;   // 1-D reference tables (read through scalar loads)
  Tab1D<float>* tab32 = nullptr;
  double* Vw = nullptr;      // [E][nq^3]  V(q) * W_q
  float* Vw_f = nullptr;
  double* W3 = nullptr;      // [nq^3]     W_q of one cell
  float* W3_f = nullptr;
  double* Minv = nullptr;    // [M]        1 / M_D
  float* Minv_f = nullptr;
  int32_t* cells_by_colour = nullptr;  // [E]
  int32_t* cell_pack = nullptr;        // [E] the same cells as i | j << 10 | k << 20
  uint32_t* cell_own = nullptr;        // [E] bit ca + 3 cb + 9 cc: the cell visits those nodes first
  // projector structure
  int32_t* node2srow = nullptr;   // [M]  support row of a DOF, -1 if none
  int32_t* srow_ptr = nullptr;    // [nsrow+1]
  int32_t* srow_atom = nullptr;   // [nent]
  int32_t* srow_coff = nullptr;   // [nent] offset of the C row in Cvals
  double* Cvals = nullptr;        // atom-major rows of C^a on support nodes
  float* Cvals_f = nullptr;
  double* Cvals_im = nullptr;     // imaginary parts (complex operators; else null)
  float* Cvals_im_f = nullptr;
  int32_t* atom_nodes = nullptr;  // concatenated support node lists (DOFs)
  int32_t* item_atom = nullptr;   // reduction work items
  int32_t* item_row0 = nullptr;   // row range inside the atom's list
  int32_t* item_row1 = nullptr;
  int32_t* item_poff = nullptr;   // offset of the item's partial block (in units of ncols)
  int32_t* item_ptr = nullptr;    // [natoms+1] items of each atom
  int32_t* fix_atom = nullptr;    // add-back work items (atom, row range), ordered by atom colour
  int32_t* fix_row0 = nullptr;
  int32_t* fix_row1 = nullptr;
  int32_t* atom_noff = nullptr;   // [natoms+1] offsets into atom_nodes
  int32_t* atom_coff = nullptr;   // [natoms]   offsets into Cvals
  int32_t* nproj = nullptr;       // [natoms]
  int32_t* poff = nullptr;        // [natoms+1] projector offsets
  int32_t* poff2 = nullptr;       // [natoms+1] offsets of nproj^2 blocks
  double* dH = nullptr;
  double* dS = nullptr;
  double* dSinv = nullptr;
  double* dSinv_im = nullptr;     // complex operators with the exact G (else null)
  int32_t* gp_ptr = nullptr;      // [natoms+1] neighbour pairs (a, b) sharing support nodes
  int32_t* gp_b = nullptr;
  int32_t* gp_off = nullptr;      // offset of G^{ab} (nproj_a x nproj_b, row-major)
  double* Gvals = nullptr;
  double* Gvals_im = nullptr;     // complex operators (else null)
  // general operators (graded mesh and / or the GGA term)
  double* geo = nullptr;          // [E][4] fx, fy, fz, det J of each cell
  float* geo_f = nullptr;
  double* vg = nullptr;           // [E][3][nq^3] W_q det J (2/h_d) V_GGA,d (GGA term)
  float* vg_f = nullptr;
  double* cscale = nullptr;       // [E] det J_e / det J (graded meshes; band-energy density)
  // [E][6] per face of a cell (x lo, x hi, y lo, y hi, z lo, z hi): the
  // lumped mass 2 w_0 h_e / 2 that the uniform tables assume for a node on
  // that face over its own w_0 (h_e + h_neighbour) / 2 (1 on uniform meshes)
  double* frho = nullptr;
  float* frho_f = nullptr;
};

}  // namespace pawfe

struct pawfe_op {
  // geometry
  int n[3];
  double L[3], h[3];
  int p, np, nq, nloc, nq3;
  int64_t M;
  int E;
  double detJ;   // det J of a cell of the uniform size box / ncell
  // graded mesh: per-axis cell boundaries (n[d] + 1 each) and per-cell det J;
  // uniform meshes keep bnd[d][i] = i h[d] and an empty cell_detJ
  bool graded = false;
  std::vector<double> bnd[3];
  std::vector<double> cell_detJ;
  // GGA term: V_GGA at the Gauss points, [E][3][nq^3]
  bool gga = false;
  std::vector<double> vgga;
  // graded or GGA: every local term runs on the general vector-ALU variants
  bool general = false;
  // host tables
  std::vector<double> gll_x, gll_w, gauss_x, gauss_w;
  std::vector<double> B, D, K1, M1, G1, W3, MD;   // G1[a][b] = sum_q w_q N_a N_b' (reference)
  // complex (k-point) operator: X is stored as interleaved (re, im) columns
  bool cplx = false;
  double kpt[3] = {0.0, 0.0, 0.0};
  std::vector<double> veff;
  // colouring
  int ncolour;
  std::vector<int32_t> colour_off;
  std::vector<int32_t> cells_by_colour;
  std::vector<int32_t> cell_colour;
  std::vector<uint32_t> cell_own;   // [E] first-visit bits per local position class
  // atoms
  int natoms;
  int npj_total, npj_max, npj2_total;
  std::vector<int32_t> nproj, poff, poff2;
  std::vector<int64_t> supp_cell_off, supp_cells, supp_node_off, supp_nodes;
  std::vector<double> Cvals;           // atom-major: atom a rows at atom_coff[a]
  std::vector<double> Cvals_im;        // imaginary parts (complex operators)
  std::vector<int32_t> atom_coff;
  std::vector<double> dH, dS, dSinv, dSinv_im;   // dSinv_im: complex operators, exact G
  std::vector<int32_t> gp_ptr, gp_b, gp_off;
  std::vector<double> Gvals, Gvals_im;
  int64_t nsrow = 0, nent = 0;
  std::vector<int32_t> node2srow, srow_ptr, srow_atom, srow_coff;
  std::vector<int32_t> item_atom, item_row0, item_row1, item_poff, item_ptr, atom_noff, atom_nodes;
  int nitems = 0;
  // atoms coloured so that atoms of one colour share no support node; the
  // add-back of C^a q_a runs one colour at a time without write conflicts
  int natom_colours = 0;
  std::vector<int32_t> fix_atom, fix_row0, fix_row1, fix_colour_off;
  int64_t item_rows_total = 0;         // sum over items of nproj (partial rows per column)
  int sinv_mode;
  pawfe::DeviceTables d;
  int32_t* d_proj_atom = nullptr;   // [npj_total] atom of each projector
  int32_t* d_proj_alpha = nullptr;  // [npj_total] index inside its atom
  int32_t* d_g2_atom = nullptr;     // [npj2_total] (atom, s, t) of each Delta entry
  int32_t* d_g2_s = nullptr;
  int32_t* d_g2_t = nullptr;
  std::vector<void*> allocations;   // every device allocation, freed at destroy
  // scratch of the stand-alone applies
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  // dense solver handle (rocBLAS handle, opaque here)
  void* blas = nullptr;
  // fork/join events of the filter's overlap of column blocks (the block
  // streams themselves are the library's, one set per device), created on
  // first use
  hipEvent_t fevent[pawfe::kMaxConcBlocks + 1] = {};
};

namespace pawfe {

// builder.cpp
pawfe_status build_host(const pawfe_op_desc* desc, pawfe_op* op);
pawfe_status upload(pawfe_op* op, hipStream_t s);
pawfe_status upload_veff(pawfe_op* op, hipStream_t s);
void free_device(pawfe_op* op);

// Host-side reference-element helpers (builder.cpp)
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w);
void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w);

}  // namespace pawfe
