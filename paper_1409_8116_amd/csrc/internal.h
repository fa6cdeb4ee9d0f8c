// Internal structures shared by the host plan layer and the device kernels.
// Not part of the public C ABI (include/mpois.h).
#pragma once
#include <cstdint>

namespace mpois {

// Real line transforms.  Forward kinds map a real line of n values to n real
// coefficients, inverse kinds map n coefficients back (all unnormalised).
//   R2HC : real DFT, half-complex output (Re X_0..X_{n/2}, Im X_{(n-1)/2}..Im X_1)
//   HC2R : inverse of R2HC times n
//   DCT2 / DCT3 / DST2 / DST3 / DCT1 / DST1 : Table 1 of the paper
//   DST4 / DCT4 : 2 sum_j x_j sin / cos(pi (j+1/2)(k+1/2)/n), the transforms of
//                 a staggered axis with a Dirichlet face and a Neumann face
enum Kind : int {
  K_R2HC = 0, K_HC2R = 1, K_DCT2 = 2, K_DCT3 = 3,
  K_DST2 = 4, K_DST3 = 5, K_DCT1 = 6, K_DST1 = 7,
  K_DST4 = 8, K_DCT4 = 9
};

constexpr int MAX_STAGES = 16;

// One Stockham stage: radix, product of the radices before it (ns), offset of
// its twiddles e^{-2 pi i r k/(ns R)} (k < ns, 1 <= r < R) and, for odd radices
// of 5 and above, of the R constants e^{2 pi i j/R} used by the codelet; and a
// reciprocal of ns for the quotients of the run-time stage loop.
struct Stage {
  int radix;
  int ns;
  int tw_off;
  int cs_off;
  unsigned ns_mul;  // floor(2^32 / ns) + 1 (0 when ns = 1): b mod ns without a division (b < 2^16)
};

// Device description of the complex DFT that one axis's line transforms use.
struct AxisDev {
  int n;          // line length (real values)
  int M;          // logical complex DFT length
  int P;          // work length: M, or the power of two of the Bluestein convolution
  int nstages;
  int bluestein;  // 1: the length-M DFT is a chirp convolution of length P
  int pad_;
  const Stage* st;    // nstages entries, device memory
  const void* tw;     // complex, working precision
  const void* pre;    // e^{-i pi k/(2n)}, k < n (DCT2/DCT3/DST2/DST3/DST4/DCT4 kinds),
                      // then entry n = e^{-i pi/(4n)}
  const void* chirp;  // e^{-i pi m^2/M}, m < M (Bluestein)
  const void* bhat;   // DFT_P of the conjugate chirp kernel, divided by P (Bluestein)
  const void* cs;     // odd-radix constants
};

// Projection step of an incompressible-flow solver on the staggered (MAC)
// grid, axes padded to three (a unit axis has no velocity component).  Face f
// of axis d lies on the low side of cell f; component d has n[d] + ext[d]
// faces along axis d (ext 0: periodic, face n is face 0; ext 1: faces 0 and
// n on the boundary) and n[e] along the other axes, in C order.  The
// gradient at a boundary face is 0 on a Neumann face (the velocity there is
// kept) and +-2 phi / h on a Dirichlet face (phi = 0 on the face).
struct ProjDev {
  void* vel[3];         // velocity components, corrected in place (null on unit axes)
  void* p;              // pressure at the cells, p += phi
  int64_t n[3];
  int64_t vs[3][3];     // element strides of component d along each axis
  int ext[3];
  int dlo[3], dhi[3];   // 1: that boundary face is Dirichlet
  double inv_h[3];
  double adt;           // alpha dt: u -= adt grad phi
  double inv_adt;       // the Poisson right-hand side is div u / adt
};

// One launch of the line-transform kernel along one axis.
struct PassArgs {
  const void* src;
  void* dst;
  int src_f64;          // element type of src: 1 double, 0 float
  int dst_f64;          // element type of dst
  int64_t nlines;       // number of lines along the axis
  int64_t inner;        // element stride along a line (product of later dims)
  int kind_f;           // transform applied first
  int kind_b;           // transform applied after the eigenvalue scaling; -1 = none
  int update;           // 1: dst <- dst + result - shift[0]  (dst is double)
  int singular;         // 1: the all-zero mode gets coefficient 0
  const double* shift;  // device scalar subtracted in update mode, or null
  const void* lam_this; // scaled eigenvalues along this axis (working precision)
  const void* lam_a;    // scaled eigenvalues of the other axes, or null
  const void* lam_b;
  int64_t nb;           // length of the axis behind lam_b
  AxisDev ax;
  // Element addressing of src and dst: element j of line l sits at
  // (l / vnb) * va + (l % vnb) * vb + j * vd.  A C-contiguous array has
  // vnb = inner, va = n * inner, vb = 1, vd = inner; a view into a larger
  // (halo-padded) array has the strides of that array.  contig: both are
  // C-contiguous (the specialised tile paths need it).
  int64_t src_vnb, src_va, src_vb, src_vd;
  int64_t dst_vnb, dst_va, dst_vb, dst_vd;
  int contig;
  // Projection step (passes along the last padded axis, C-contiguous phi):
  // proj_load, the source is div(vel) / adt formed from proj.vel as it is
  // read; proj_store, the pass also adds phi to proj.p and corrects the
  // velocity component along the pass axis.
  int proj_load;
  int proj_store;
  ProjDev proj;
};

// One launch of the line-transform kernel over many grids.
struct BatchPassArgs {
  const PassArgs* args;       // per-grid pass description (src/dst/update fields ignored)
  const int* tile_prob;       // per block: grid index
  const int* tile_idx;        // per block: tile index within that grid
  const void* const* src_tab; // per-grid source array
  void* const* dst_tab;       // per-grid destination array
  int src_f64, dst_f64, update;
  int shift_stride;           // doubles between consecutive grids' scalars
  const double* shift_base;   // first grid's gauge shift (singular grids only), or null
};

// Stencil residual over a (n0, n1, n2) box, all axes described by a closure.
enum Closure : int { C_NONE = 0, C_PER = 1, C_DV = 2, C_DS = 3, C_NV = 4, C_NS = 5 };

struct ResidArgs {
  const double* phi;
  const double* g;
  void* r;              // output residual (or null), float or double
  int r_f64;
  int64_t n[3];
  int64_t ps[3];        // element strides of phi per axis (C-contiguous: n1 n2, n2, 1)
  int64_t gs[3];        // element strides of g (r is always C-contiguous)
  int clo[3];           // closure at the low end of each axis
  int chi[3];           // closure at the high end
  double inv_h2[3];
  double shift;         // Helmholtz sigma: r = g - m_g - (L_h - sigma) phi
  const double* mg;     // device scalar subtracted from g (or null)
  double* partials;     // 4 per block: sum w phi, sum w g, sum r^2, sum (g-mg)^2
  int singular;         // every axis periodic or Neumann
};

// Residual over many grids in one launch: block b handles grid blk_prob[b]
// as its block (b - blk_start[grid]) of blk_count[grid].
struct BatchResidArgs {
  const ResidArgs* args;      // per grid (phi/g/r/mg/partials fields ignored)
  const int* blk_prob;
  const int* blk_start;       // per grid: first block
  const int* blk_count;       // per grid: number of blocks
  const void* const* phi_tab;
  const void* const* g_tab;
  void* const* r_tab;         // or null: no residual output
  int r_f64;
  int use_mg;                 // subtract scalars[grid].S_MG from g on singular grids
  double* scalars;            // S_COUNT per grid
  double* partials;           // 4 per block
};

// Reduced scalars kept on the device.
enum Scalar : int {
  S_WPHI = 0,   // sum w phi
  S_WG = 1,     // sum w g
  S_R2 = 2,     // sum r^2
  S_G2 = 3,     // sum (g - m_g)^2
  S_SHIFT = 4,  // sum w phi / sum w
  S_MG = 5,     // sum w g / sum w
  S_COUNT = 8
};

}  // namespace mpois
