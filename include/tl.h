/*
 * tl.h - C ABI of the MI355X (gfx950) lattice core-Hamiltonian library.
 *
 * Method: Khoromskaia & Khoromskij, "Tensor numerical approach to linearized
 * Hartree-Fock equation for lattice-type and periodic systems"
 * (arXiv:1408.3839).  The library assembles the Galerkin core Hamiltonian
 * H = T - V_c and the mass matrix S of a Gaussian basis replicated over an
 * (L1,L2,L3) lattice, with every basis function and the Newton potential held
 * as separable 1D vectors on a global 3D grid, and diagonalises the periodic
 * case through the block-circulant structure.
 *
 * Conventions shared by every call
 *   - All array arguments named *_dev are device pointers (HBM) owned by the
 *     caller; the library never allocates, frees or retains them.  All other
 *     pointers (inside tl_system) are host pointers read during the call only.
 *   - Every call is asynchronous on `stream` (a hipStream_t, passed as void*;
 *     NULL = the default stream).  It validates its arguments, enqueues its
 *     kernels and returns; results are valid once the stream is synchronised.
 *   - Return value: TL_OK (0) or a negative tl_status.  On error nothing is
 *     enqueued and tl_last_error() returns a message for the calling thread.
 *   - Layout: row-major, FP64.  Complex values are interleaved (re, im) pairs.
 *   - Numerical failures inside a batched eigensolve never fail the call;
 *     they are reported per problem in an `info` array.
 */
#ifndef TL_H
#define TL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tl_status;
#define TL_OK 0
#define TL_EINVAL (-1)         /* invalid argument (see tl_last_error)          */
#define TL_EUNSUPPORTED (-2)   /* valid request outside what this build covers  */
#define TL_EHIP (-3)           /* a HIP runtime call failed                     */
#define TL_EWORKSPACE (-4)     /* workspace argument smaller than required      */

typedef enum {
  TL_FP64 = 0,        /* 1D contractions in FP64 (MFMA f64)                          */
  TL_FP32 = 1,        /* 1D contractions in FP32 (MFMA f32), FP64 chunk sums         */
  TL_SPLIT_BF16 = 2,  /* operands split into bf16 slices, FP32 MFMA accumulation     */
  TL_SPLIT_FP16 = 3   /* operands split into fp16 slices, FP32 MFMA accumulation     */
} tl_precision;

#define TL_MODE_PERIODIC 0   /* first block column of the 3-level block circulant */
#define TL_MODE_BOX 1        /* full matrices of an open-boundary chain           */

#define TL_MAX_M0 32
#define TL_MAX_SITES 16
#define TL_MAX_R 64

/*
 * Problem description (host memory).  Dimension l in {0,1,2} is x, y, z.
 *  periodic[l] = 1: torus of L[l] cells of length a[l]; nodes x_i = i*h,
 *     n[l] = L[l]*cell_nodes[l], cell_nodes[l] = a[l]/h (an integer).
 *  periodic[l] = 0: open box, nodes x_i = x0[l] + i*h, homogeneous Dirichlet
 *     conditions outside the n[l] nodes (Sec. 3.4).
 *  mode TL_MODE_PERIODIC: nuc_pos/nuc_Z are the n_nuc sites of the unit cell
 *     (offsets from the cell origin, k*a for cell k), at most TL_MAX_SITES;
 *     in periodic dims the offsets must be multiples of h.  K[l] is the image
 *     range -K..K of the lattice sum restricted to the central cell
 *     (Sec. 4.1, eq. (EwaldSumP)).
 *  mode TL_MODE_BOX: nuc_pos/nuc_Z list every nucleus (absolute positions);
 *     the L[0] cells of a chain along x carry the basis, cell c at
 *     x = box_origin0 + c*a[0], y = z = 0.  All three dims must be open.
 *  Basis function mu of a cell (m0 <= TL_MAX_M0): centre cell origin +
 *     fn_center[3*mu..], 1D factors fn_coef[3*mu+l] (x-A_l)^fn_l[3*mu+l]
 *     exp(-fn_alpha[mu] (x-A_l)^2), fn_l in {0,1}.
 *  Newton kernel: 1/rho ~ sum_{q<R} w_q exp(-t_q^2 rho^2) (Sec. 3.2,
 *     eq. (sinc_general)).
 */
typedef struct {
  int mode;
  int L[3];
  int periodic[3];
  int n[3];
  int cell_nodes[3];
  int K[3];
  double h;
  double x0[3];
  double a[3];
  double box_origin0;
  int n_nuc;
  const double* nuc_pos;   /* [n_nuc][3] */
  const double* nuc_Z;     /* [n_nuc]    */
  int m0;
  const double* fn_center; /* [m0][3] */
  const int* fn_l;         /* [m0][3] */
  const double* fn_alpha;  /* [m0]    */
  const double* fn_coef;   /* [m0][3] */
  int R;
  const double* t_q;       /* [R] */
  const double* w_q;       /* [R] */
} tl_system;

/* Library identification and the thread-local text of the last error. */
const char* tl_version(void);
const char* tl_status_string(tl_status s);
const char* tl_last_error(void);

/*
 * Sizes (in elements, not bytes) of the arrays exchanged for a system.
 *   basis_rows[l]   rows of the sampled basis on dim l: m0, or L[0]*m0 on
 *                   dim 0 in box mode.
 *   basis_elems     sum_l basis_rows[l]*n[l] (one array each for G, AG, SG;
 *                   dim l starts at offset sum_{e<l} basis_rows[e]*n[e]).
 *   pot_terms       canonical rank of the potential: R times the number of
 *                   groups of nuclei sharing their (y,z) position.
 *   pot_elems       sum_l pot_terms*n[l] (dim l at offset pot_terms*sum_{e<l} n[e]).
 *   block_elems     periodic: L1*L2*L3*m0*m0 (one real array each for H, S);
 *                   box: (L[0]*m0)^2.
 */
typedef struct {
  int64_t basis_rows[3];
  int64_t basis_elems;
  int64_t pot_terms;
  int64_t pot_elems;
  int64_t block_elems;
} tl_sizes;
tl_status tl_query_sizes(const tl_system* sys, tl_sizes* out);

/* Workspace (bytes of device memory, 256-byte aligned by the caller) that
 * tl_lattice_sum_potential and tl_assemble_core_hamiltonian_block need. */
tl_status tl_potential_workspace_bytes(const tl_system* sys, size_t* bytes);
tl_status tl_assemble_workspace_bytes(const tl_system* sys, tl_precision prec,
                                      int n_slices, size_t* bytes);
tl_status tl_block_fft_workspace_bytes(int L1, int L2, int L3, int m0, int batch,
                                       size_t* bytes);

/*
 * tl_build_basis - nodal samples of the basis and its FEM images
 * (Sec. 3.4, eq. (Gaus pwl) and the 1D matrices A = (1/h) tridiag(-1,2,-1),
 * S = (h/6) tridiag(1,4,1)).
 *   G_dev[row][i]  = g_row(x_i), periodised over the torus in periodic dims
 *                    (sum over images within exp(-46) of the peak),
 *   AG_dev = A g, SG_dev = S g (circulant on a torus, Dirichlet in a box).
 * Each array holds basis_elems doubles.  Periodic mode: the rows are the m0
 * functions of cell 0; box mode, dim 0: row c*m0+mu is function mu of cell c.
 */
tl_status tl_build_basis(const tl_system* sys, double* G_dev, double* AG_dev, double* SG_dev,
                         void* stream);

/*
 * tl_lattice_sum_potential - canonical 1D vectors of the lattice-summed
 * Newton potential (Sec. 3.2 eqs. (galten), (core_tens), (EwaldTensorGl);
 * Sec. 4.1 eq. (EwaldSumP)).  For term t = g*R + q (g = group of nuclei with
 * equal (y,z), q = quadrature node):
 *   P_dev[l][t][i] = prod over l of these factors gives sum_nu Z_nu w_q
 *   exp-sum image of the cell-averaged kernel; w_q and Z_nu sit in dim 0.
 *   Periodic dims: image sum k = -K..K of cell integrals
 *   int_cell exp(-t_q^2 (y - o - k a)^2) dy evaluated on the central cell and
 *   replicated with period a (entries of the "master" vector on the
 *   accompanying grid, formed where they are summed); box dims: one factor
 *   per nucleus.
 * P_dev holds pot_elems doubles.  tl_potential_workspace_bytes reports 0
 * (no scratch memory is used); ws_dev may then be NULL.
 */
tl_status tl_lattice_sum_potential(const tl_system* sys, double* P_dev, void* ws_dev,
                                   size_t ws_bytes, void* stream);

/*
 * tl_build_basis_and_potential - tl_build_basis and tl_lattice_sum_potential
 * in one call, with the arguments and outputs of the two (G_dev, AG_dev,
 * SG_dev: basis_elems doubles each; P_dev: pot_elems doubles; ws as for the
 * potential).  The results are bit-identical to the two calls in sequence.
 * For a system periodic in dim 0 with m0 <= 8 both steps share one kernel
 * launch (they are independent); otherwise the two launches run in order.
 * Errors: TL_EINVAL for an invalid system or a null output array.
 */
tl_status tl_build_basis_and_potential(const tl_system* sys, double* G_dev, double* AG_dev,
                                       double* SG_dev, double* P_dev, void* ws_dev,
                                       size_t ws_bytes, void* stream);

/*
 * tl_assemble_core_hamiltonian_block - Galerkin matrices from 1D inner
 * products (proof of Lemma 3.1, eq. (nuc_potMatrTot); Sec. 3.4 A_3; Lemma 4.1
 * eqs. (BC-Core), (BC-mass), (BC-Laplace)):
 *   C_l[t][mu][nu][s] = sum_i g_mu(x_i - s a_l) p_t(x_i) g_nu(x_i)
 *   D_l, M_l likewise with A g_nu, S g_nu in place of p_t g_nu,
 *   V = sum_t prod_l C_l,  T = 1/2 (D1 M2 M3 + M1 D2 M3 + M1 M2 D3),
 *   S = M1 M2 M3,  H = T - V.
 * Periodic mode: H_dev, S_dev = generating blocks (first block column)
 *   [k1][k2][k3][mu][nu], A_k[mu][nu] = <g_(mu, cell k) | op | g_(nu, cell 0)>,
 *   only shifts 0..L/2 are contracted; A_{-k} = A_k^T fills the rest.
 * Box mode: H_dev, S_dev = full (L0*m0)^2 matrices, row c*m0+mu.
 * prec selects the arithmetic of the 1D contractions; the combination over
 * terms and dimensions is FP64 in every mode.  n_slices is used by the split
 * modes (2..6 slices per operand for TL_SPLIT_FP16, 2..7 for TL_SPLIT_BF16;
 * 0 takes 5 and 6), ignored otherwise.
 * Box mode runs the x contraction in FP64 or a split mode (TL_FP32 gives
 * TL_EUNSUPPORTED); its y and z factors (m0 x m0 per term) are FP64.
 * Inputs: the arrays filled by tl_build_basis and tl_lattice_sum_potential.
 */
tl_status tl_assemble_core_hamiltonian_block(const tl_system* sys, const double* G_dev,
                                             const double* AG_dev, const double* SG_dev,
                                             const double* P_dev, tl_precision prec,
                                             int n_slices, double* H_dev, double* S_dev,
                                             void* ws_dev, size_t ws_bytes, void* stream);

/*
 * tl_assemble_kblocks - the k-blocks Hbar_k, Sbar_k of a periodic system
 * straight from the 1D contractions, with the lattice DFT taken factor by
 * factor (Theorem on the tensor-structured FFT diagonalisation, Sec. 2;
 * Proposition on low-rank Fourier coefficients):
 *   Chat_l[t][mu][nu](k) = sum_{d=0}^{L_l-1} C_l[t][mu][nu][d] w_l^(k d),
 *   w_l = exp(-2 pi i / L_l), C_l[mu][nu][-s] = C_l[nu][mu][s] on the torus,
 *   Vbar_k = sum_t prod_l Chat_l[t](k_l), Tbar_k and Sbar_k likewise from
 *   the D and M factors, Hbar_k = Tbar_k - Vbar_k.
 * The result equals tl_assemble_core_hamiltonian_block followed by
 * tl_block_fft (up to rounding), without the real-space block column.
 *   Hk_dev, Sk_dev: [L1][L2][L3][m0][m0] complex (interleaved re, im), the
 *   layout tl_block_fft writes and tl_batched_heigh reads.
 *   prec, n_slices, inputs: as tl_assemble_core_hamiltonian_block.
 *   ws_dev: tl_assemble_kblocks_workspace_bytes bytes (the contraction's
 *   workspace plus (T+2) m0^2 L_l complex values per transformed dim).
 * Errors: TL_EUNSUPPORTED for box mode or a periodic L_l above 2048 (the
 * block FFT route takes those), TL_EWORKSPACE, TL_EINVAL as for assembly.
 */
tl_status tl_assemble_kblocks_workspace_bytes(const tl_system* sys, tl_precision prec,
                                              int n_slices, size_t* bytes);
tl_status tl_assemble_kblocks(const tl_system* sys, const double* G_dev, const double* AG_dev,
                              const double* SG_dev, const double* P_dev, tl_precision prec,
                              int n_slices, double* Hk_dev, double* Sk_dev, void* ws_dev,
                              size_t ws_bytes, void* stream);

/*
 * tl_assemble_core_hamiltonian_block_noalloc - the same assembly for callers
 * that cannot allocate or pass device memory for scratch (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *   Arguments, outputs and results as tl_assemble_core_hamiltonian_block
 *   (bit-identical outputs; the same kernels), without ws_dev/ws_bytes: the
 *   scratch is a static device array of 32 MiB that each device the library
 *   runs on holds until the process ends.  Calls no hipMalloc/hipFree.
 *   The device is the current one (hipGetDevice) at the call; its scratch
 *   address is looked up on the first call on that device.
 *   Errors: those of tl_assemble_core_hamiltonian_block, and TL_EUNSUPPORTED
 *   when the system needs more scratch than 32 MiB
 *   (tl_assemble_workspace_bytes tells); nothing is enqueued then.
 *   Every call on one device shares that device's scratch: calls that
 *   overlap on one device (different streams, or different threads) race.
 *   Calls on one stream are ordered and safe.
 */
tl_status tl_assemble_core_hamiltonian_block_noalloc(const tl_system* sys, const double* G_dev,
                                                     const double* AG_dev, const double* SG_dev,
                                                     const double* P_dev, tl_precision prec,
                                                     int n_slices, double* H_dev, double* S_dev,
                                                     void* stream);

/*
 * tl_set_contraction_events - profiling hook: when both are non-NULL, the
 * assembly and batch calls made afterwards by the calling thread attach
 * start_event and stop_event (hipEvent_t, created with timing) to the launch
 * of the 1D-contraction kernel itself (hipExtLaunchKernel), so
 * hipEventElapsedTime gives that kernel's duration on its stream.  NULL,
 * NULL switches the hook off.  The events stay owned by the caller.
 */
tl_status tl_set_contraction_events(void* start_event, void* stop_event);

/*
 * tl_set_stage_events - the same profiling hook for one stage of the path:
 *   TL_STAGE_CONTRACTION  the 1D-contraction launch (as above),
 *   TL_STAGE_LATTICE_SUM  the lattice-sum launch of tl_lattice_sum_potential
 *                         (torus and open transverse dims) and of the batch,
 *   TL_STAGE_FFT          the LDS block-FFT launch of tl_block_fft and of the
 *                         batch.
 * Events are per calling thread and stay owned by the caller; NULL, NULL
 * switches the stage's hook off.  TL_EINVAL for an unknown stage or a
 * single null event.
 */
#define TL_STAGE_CONTRACTION 0
#define TL_STAGE_LATTICE_SUM 1
#define TL_STAGE_FFT 2
#define TL_STAGE_COUNT 3
tl_status tl_set_stage_events(int stage, void* start_event, void* stop_event);

/*
 * tl_block_fft - Fourier block-diagonalisation of 3-level block-circulant
 * matrices (Lemma 2.2 eq. (DiagMLcirc); Appendix, Proposition on
 * block-circulant diagonalisation):
 *   out[b][j1][j2][j3] = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) in[b][k1][k2][k3],
 *   w_l = exp(-2 pi i / L_l), for every m0 x m0 entry, for each of `batch`
 *   real input block columns.  in_dev: batch*L1*L2*L3*m0*m0 doubles;
 *   out_dev: the same count of complex values (2x doubles).
 * ws_dev: tl_block_fft_workspace_bytes (0 when at most one L_l exceeds 1).
 */
tl_status tl_block_fft(const double* in_dev, int L1, int L2, int L3, int m0, int batch,
                       double* out_dev, void* ws_dev, size_t ws_bytes, void* stream);

/*
 * tl_batched_heigh - eigenvalues (and optionally eigenvectors) of `count`
 * Hermitian-definite pencils (Hbar_j - lambda Sbar_j) u = 0 of order m0
 * (Sec. 4.2 eq. (HF-FSpace-Block); Proposition eq. (lambdAbc)).
 *   H_dev, S_dev: [count][m0][m0] complex (S_dev may be NULL: standard problem).
 *   evals_dev: [count][m0] ascending.  evecs_dev (nullable): [count][m0][m0]
 *   complex, column m = eigenvector of evals[m], normalised u^H Sbar u = 1.
 *   info_dev: [count] int, 0 = converged, k > 0 = Sbar not positive definite
 *   at pivot k (evals set to NaN), -1 = Jacobi iteration did not converge.
 * Method: Cholesky Sbar = L L^H, C = L^-1 Hbar L^-H, then for m0 <= 16
 * without eigenvectors (evecs_dev NULL) a complex Householder reduction of C
 * to a real tridiagonal and Sturm bisection (one wave per block for m0 <= 8,
 * 256 threads above), otherwise cyclic parallel complex Jacobi with
 * u = L^-H v.  1 <= m0 <= TL_MAX_M0.
 */
tl_status tl_batched_heigh(const double* H_dev, const double* S_dev, int count, int m0,
                           double* evals_dev, double* evecs_dev, int* info_dev, void* stream);

/*
 * tl_bloch_vectors - eigenvectors of the full block-circulant pencil from
 * those of its k-blocks (Appendix, Proposition on block-circulant
 * diagonalisation, eq. (eigvecA)): with F = F_L1 x F_L2 x F_L3 unitary,
 *   U_(j,m) = (F^* x I_m0) (e_j x u_(j,m)),
 *   U_(j,m)[c][mu] = L^(-1/2) exp(2 pi i sum_l j_l c_l / L_l) u_(j,m)[mu],
 *   L = L1 L2 L3, j and c flat indices [j1][j2][j3], [c1][c2][c3].
 *   evecs_dev: [L][m0][m0] complex, column m = eigenvector m of block j (the
 *   layout tl_batched_heigh writes; S-normalised vectors there give
 *   U^H S U = 1 for the full mass matrix).
 *   states_dev: n_states int32 in device memory, flat state indices j*m0 + m;
 *   an index outside [0, L*m0) yields a NaN vector.
 *   out_dev: [n_states][L][m0] complex (interleaved re, im), row r = state r.
 * Errors: TL_EINVAL for sizes out of range or a null array with n_states > 0.
 */
tl_status tl_bloch_vectors(const double* evecs_dev, int L1, int L2, int L3, int m0,
                           const int* states_dev, int n_states, double* out_dev, void* stream);

/*
 * tl_bloch_orbital_factors - the orbital of a Bloch state on the grid as a
 * canonical tensor of rank m0 (eq. (eigvecA) with the separable basis of
 * Sec. 3.4): psi(x) = sum_mu w_mu prod_d phi^d_mu(x_d), with
 *   w_mu = L^(-1/2) u_(j,m)[mu],
 *   phi^d_mu(x_i) = sum_(c=0)^(L_d-1) exp(2 pi i j_d c / L_d) g^d_mu(x_i - c a_d)
 * (the periodised samples of tl_build_basis read c * cell_nodes_d nodes back
 * on the torus; an open dim has phi = g).  Periodic systems only.
 *   G_dev: the basis samples of tl_build_basis (basis_elems doubles).
 *   evecs_dev, states_dev: as for tl_bloch_vectors.
 *   coef_dev: [n_states][m0] complex; factors_dev: [n_states][basis_elems]
 *   complex, dim d at offset basis_off(d) = sum_(e<d) m0 n_e, row mu of n_d.
 *   An index outside [0, L m0) yields NaN.
 * Errors: TL_EINVAL (system, null array), TL_EUNSUPPORTED (box mode).
 */
tl_status tl_bloch_orbital_factors(const tl_system* sys, const double* G_dev,
                                   const double* evecs_dev, const int* states_dev, int n_states,
                                   double* coef_dev, double* factors_dev, void* stream);

/*
 * tl_chain_orbital_factors - the open chain's orbitals on the grid as
 * canonical tensors of rank m0 (Sec. 3.4's separable basis; the transverse
 * factors are the same for every cell): psi = sum_mu phi^x_mu x g^y_mu x g^z_mu,
 * phi^x_mu(x_i) = sum_c U[c m0 + mu] g^x_(c,mu)(x_i).  Box systems only.
 *   G_dev: the box-mode basis samples of tl_build_basis.
 *   evecs_dev: n_states rows of L m0 doubles (the layout tl_dense_gen_eigh_lowest
 *   writes, cell-major, function-minor).
 *   factors_dev: [n_states][m0 (n0 + n1 + n2)] doubles, dim d at offset
 *   m0 sum_(e<d) n_e, row mu of n_d.
 * Errors: TL_EINVAL (system, null array), TL_EUNSUPPORTED (periodic mode).
 */
tl_status tl_chain_orbital_factors(const tl_system* sys, const double* G_dev,
                                   const double* evecs_dev, int n_states, double* factors_dev,
                                   void* stream);

/*
 * Symmetric block-Toeplitz matrices (Sec. 2, Definition of the block
 * Toeplitz class; Appendix eq. (block_SToepl)), as the open chain's matrices
 * are up to a boundary defect (Sec. 3.3): A = BToepl_s{A_0..A_{L-1}}, block
 * (r, c) = A_{r-c} (r >= c), A_{c-r}^T (r < c).  Products with A go through
 * the double-size block-circulant embedding (Remark on block Toeplitz
 * matrices): C_k = A_k (k < L), C_L = 0, C_{2L-k} = A_k^T, diagonalised by the
 * block DFT over 2L cells, O(m0^2 L log L + m0^2 nvec L) per product instead
 * of (L m0)^2 nvec.
 *   tl_btoepl_workspace_bytes  workspace for (L, m0, nvec): the 2L k-blocks
 *       of C and the transforms of one block of nvec vectors.
 *   tl_btoepl_setup   A_dev: [L][m0][m0] (A_0 symmetric); forms the k-blocks
 *       of C in the workspace (once per matrix; the workspace then serves
 *       every product with that matrix and nvec).
 *   tl_btoepl_matvec  Y = A X, X_dev and Y_dev [L][m0][nvec] (cell, function,
 *       vector), FP64.
 *   tl_btoepl_power   the power method for the senior eigenvalue (largest in
 *       magnitude), the Remark's use: iters times y = A x,
 *       lambda[it] = (x . y) / (x . x), x = y / |y|.  x_dev: start vector in,
 *       last iterate out; y_dev: scratch; both L*m0 doubles; lambda_dev:
 *       iters doubles.  Workspace and setup as for nvec = 1.
 * Limits: 1 <= L <= 2048 (2L on the block FFT; lengths 2L with a prime factor
 * above 7 use Bluestein and need 4L - 1 <= 4096), 1 <= m0 <= TL_MAX_M0,
 * 1 <= nvec <= 1024.  Errors: TL_EINVAL, TL_EUNSUPPORTED (no transform plan).
 */
tl_status tl_btoepl_workspace_bytes(int L, int m0, int nvec, size_t* bytes);
tl_status tl_btoepl_setup(const double* A_dev, int L, int m0, int nvec, void* ws_dev,
                          size_t ws_bytes, void* stream);
tl_status tl_btoepl_matvec(const double* X_dev, double* Y_dev, int L, int m0, int nvec,
                           void* ws_dev, size_t ws_bytes, void* stream);
tl_status tl_btoepl_power(int L, int m0, int iters, double* x_dev, double* y_dev,
                          double* lambda_dev, void* ws_dev, size_t ws_bytes, void* stream);

/*
 * Multilevel block-Toeplitz products (the recursive Definition of the d-level
 * class; the Remark's double-size embedding at each level): A over
 * L1 x L2 x L3 cells, block (r, c) = B(r - c) for cells r, c flattened as
 * [r1][r2][r3], through the block circulant C over 2L1 x 2L2 x 2L3 cells
 * (a level with L_l = 1 stays 1) and a 3D block DFT.
 *   tl_btoepl3_workspace_bytes  workspace for (L, m0, nvec).
 *   tl_btoepl3_setup  B_dev: [2L1-1][2L2-1][2L3-1][m0][m0], shift d at index
 *       d + L - 1 per level (any blocks: the symmetric class of the paper has
 *       B(-d) = B(d)^T); forms C's k-blocks in the workspace.
 *   tl_btoepl3_matvec  Y = A X, X_dev and Y_dev [L1][L2][L3][m0][nvec] FP64.
 * Limits: at most 4096 embedded cells; with two or more levels each doubled
 * length must be 7-smooth (one level may use Bluestein as in the one-level
 * product); 1 <= m0 <= TL_MAX_M0, 1 <= nvec <= 1024.
 * Errors: TL_EINVAL, TL_EWORKSPACE, TL_EUNSUPPORTED (no transform plan).
 */
tl_status tl_btoepl3_workspace_bytes(int L1, int L2, int L3, int m0, int nvec, size_t* bytes);
tl_status tl_btoepl3_setup(const double* B_dev, int L1, int L2, int L3, int m0, int nvec,
                           void* ws_dev, size_t ws_bytes, void* stream);
tl_status tl_btoepl3_matvec(const double* X_dev, double* Y_dev, int L1, int L2, int L3, int m0,
                            int nvec, void* ws_dev, size_t ws_bytes, void* stream);
/* tl_btoepl3_power: the power method of the Remark on the multilevel
 * product, as tl_btoepl_power (x_dev, y_dev: L1 L2 L3 m0 doubles; workspace
 * and set-up for nvec = 1). */
tl_status tl_btoepl3_power(int L1, int L2, int L3, int m0, int iters, double* x_dev,
                           double* y_dev, double* lambda_dev, void* ws_dev, size_t ws_bytes,
                           void* stream);

/*
 * tl_btoepl_lowest - the nev lowest eigenpairs of the symmetric-definite
 * pencil T_H u = lambda T_S u of two symmetric block-Toeplitz matrices given
 * by their first block columns (the iterative route for boxes too large for
 * the full eigensolver, Sec. 3.3's closing remark, on the embedded product of
 * the Remark on block Toeplitz matrices).  LOBPCG with a block of nb vectors,
 * preconditioned by the inverse of the shifted Strang block circulant of the
 * pencil (its k-blocks Hhat_j - sigma Shat_j, sigma = the circulant pencil's
 * lowest eigenvalue minus `shift`, through the block DFT over L cells).
 *   H_dev, S_dev: [L][m0][m0] doubles, device (A_0 symmetric); T_S must be
 *     positive definite, and so must every k-block Shat_j of its circulant.
 *   nev <= nb <= 21, 3 nb <= L m0.  A few guard vectors (nb > nev) speed up
 *     the convergence of the highest wanted pairs.
 *   max_iter: iteration limit; tol: relative residual target
 *     |T_H x - lambda T_S x| / ((|T_H| + |lambda| |T_S|) |x|), the norms
 *     bounded by the sums over k of the largest row and column sums of |A_k|.
 *   shift: sigma below the circulant minimum; <= 0 takes the larger of
 *     1e-4 max(1, |lambda_min|) and 10 times the estimated finite-size offset
 *     of the pencil's lowest eigenvalue (a quarter of the gap between the two
 *     smallest k-block minima).
 *   x0_dev (nullable): start block [L m0][nb]; NULL draws it from a fixed seed.
 *   evals_dev: nev doubles, ascending; evecs_dev (nullable): [L][m0][nev],
 *     T_S-normalised; resid_dev (nullable): the nev relative residuals,
 *     recomputed from fresh products at the end.
 *   iters, nconv (host): iterations run, and how many of the nev pairs meet
 *     tol (nconv < nev: not converged within max_iter; the outputs are the
 *     last iterate).
 * The call synchronises `stream` (the iteration is steered by residual norms
 * read back every step).  Limits: 1 <= L <= 2048 as for the product, m0 <=
 * TL_MAX_M0.  Errors: TL_EINVAL (arguments; a circulant k-block that is not
 * definite; a Rayleigh-Ritz basis that lost rank), TL_EWORKSPACE,
 * TL_EUNSUPPORTED (no transform plan for L).
 */
tl_status tl_btoepl_lowest_workspace_bytes(int L, int m0, int nb, size_t* bytes);
/* tl_btoepl3_lowest: the same solver for a pencil of symmetric multilevel
 * block-Toeplitz matrices over L1 x L2 x L3 cells (blocks for every shift as
 * for tl_btoepl3_setup, with B(-d) = B(d)^T), on the multilevel product; the
 * preconditioner is the shifted Strang circulant over the L1 x L2 x L3
 * lattice (at a half-period shift the mean of both blocks).  Vectors
 * [L1][L2][L3][m0][nev]; limits of the multilevel product (at most 4096
 * embedded cells). */
tl_status tl_btoepl3_lowest_workspace_bytes(int L1, int L2, int L3, int m0, int nb,
                                            size_t* bytes);
tl_status tl_btoepl3_lowest(const double* H_dev, const double* S_dev, int L1, int L2, int L3,
                            int m0, int nev, int nb, int max_iter, double tol, double shift,
                            const double* x0_dev, double* evals_dev, double* evecs_dev,
                            double* resid_dev, int* iters, int* nconv, void* ws_dev,
                            size_t ws_bytes, void* stream);
tl_status tl_btoepl_lowest(const double* H_dev, const double* S_dev, int L, int m0, int nev,
                           int nb, int max_iter, double tol, double shift, const double* x0_dev,
                           double* evals_dev, double* evecs_dev, double* resid_dev, int* iters,
                           int* nconv, void* ws_dev, size_t ws_bytes, void* stream);

/*
 * tl_dense_gen_eigh_lowest - the k lowest eigenpairs of the full symmetric
 * pencil H u = lambda S u, S positive definite (the open-boundary chain's
 * core Hamiltonian and mass matrix, Sec. 5's full eigensolver; Sec. 2.1
 * eq. (HF-FSpace) with C^T S C = I).
 *   H_dev, S_dev: N x N row-major doubles, device, both triangles stored
 *     (the layout tl_assemble_core_hamiltonian_block writes in box mode);
 *     read only.
 *   evals_dev: k doubles, ascending.
 *   evecs_dev (nullable): k x N row-major doubles, row m = eigenvector of
 *     evals[m], normalised u^T S u = 1 (sign arbitrary).  NULL skips the
 *     eigenvector stages.
 *   info_dev: one int: 0 = ok; j > 0 = S not positive definite at pivot j
 *     (the outputs are then meaningless but finite); -2 = eigenvectors of
 *     a numerically degenerate cluster could not be separated.
 *   ws_dev: tl_dense_gen_eigh_workspace_bytes(N, k) bytes, device.
 * Limits: 1 <= N <= 7680, 1 <= k <= min(N, 64).
 * Method (FP64 throughout): Cholesky S = L L^T, C = L^-1 H L^-T,
 * Householder tridiagonalisation, Sturm multisection for the k lowest
 * eigenvalues, inverse iteration + Cholesky-QR for the eigenvectors,
 * back-transformation.  Asynchronous on `stream`; allocates nothing.
 */
tl_status tl_dense_gen_eigh_workspace_bytes(int N, int k, size_t* bytes);

/*
 * tl_set_dense_eigh_events - profiling hook: with count = 6, the
 * tl_dense_gen_eigh_lowest calls made afterwards by the calling thread
 * record events[i] (hipEvent_t) on their stream at the stage boundaries:
 * 0 before the Cholesky factorisation, 1 after L and L^-1, 2 after
 * C = L^-1 H L^-T, 3 after the tridiagonalisation, 4 after the eigenvalues,
 * 5 at the end.  count = 0 switches the hook off.  Events stay caller-owned.
 */
tl_status tl_set_dense_eigh_events(void* const* events, int count);
tl_status tl_dense_gen_eigh_lowest(const double* H_dev, const double* S_dev, int N, int k,
                                   double* evals_dev, double* evecs_dev, int* info_dev,
                                   void* ws_dev, size_t ws_bytes, void* stream);

/*
 * Batched path (many periodic (L,1,1) lattices of uneven L and m0): the
 * whole chain basis -> potential -> assembly -> block FFT -> k-block
 * eigensolves with ONE launch per stage for the whole batch.
 *
 *   tl_batch_plan_create  sizes every buffer for `count` systems (host only).
 *   tl_batch_write_descriptor  writes, into caller host memory of
 *       plan.desc_bytes bytes, every instance's launch arguments with device
 *       addresses inside the caller's buffers; the caller copies it to device
 *       memory once.  Buffers (device, caller-owned, contiguous per instance
 *       in the order of `systems`):
 *         G, AG, SG   basis_elems doubles each
 *         P           pot_elems doubles
 *         HS          hs_elems doubles: per instance H then S (block column)
 *         HSbar       2*hs_elems doubles: per instance Hbar then Sbar (complex)
 *         evals       eval_elems doubles: per instance [L][m0] ascending
 *         info        kblocks ints (as tl_batched_heigh)
 *         ws          ws_bytes bytes of workspace
 *   tl_batch_run  enqueues the stages on `stream`; needs the host copy of
 *       the descriptor (launch geometry) and its device copy (arguments).
 *       Allocates nothing and copies nothing: capturable in a HIP graph.
 * want_blocks is the tiling target of the contraction (workgroups per
 * instance; 0 = library default) and plan.tile_edge the largest tile edge of
 * the FP64 contraction (64 or 32; an instance whose tiles do not fit the LDS
 * budget takes the smaller edge): the parameters the autotuner chooses.
 * tl_batch_write_descriptor returns TL_EINVAL for another tile_edge.
 * Same arithmetic per instance as the single-system calls (bitwise equal
 * for equal want_blocks).
 */
#define TL_MAX_BATCH 512
typedef struct {
  int count, precision, n_slices, want_blocks;
  int max_m0, max_len;
  int64_t basis_elems, pot_elems, hs_elems, eval_elems, kblocks;
  size_t ws_bytes, desc_bytes;
  int tile_edge;  /* FP64 contraction tile edge, 64 (default) or 32; may be
                     changed between plan creation and descriptor writing */
} tl_batch_plan;

typedef struct {
  double* G;
  double* AG;
  double* SG;
  double* P;
  double* HS;
  double* HSbar;
  double* evals;
  int* info;
  void* ws;
} tl_batch_buffers;

tl_status tl_batch_plan_create(const tl_system* systems, int count, tl_precision prec,
                               int n_slices, int want_blocks, tl_batch_plan* out);
tl_status tl_batch_write_descriptor(const tl_system* systems, int count,
                                    const tl_batch_plan* plan, const tl_batch_buffers* buffers,
                                    void* host_desc, size_t desc_bytes);
tl_status tl_batch_run(const tl_batch_plan* plan, const void* host_desc, const void* desc_dev,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TL_H */
