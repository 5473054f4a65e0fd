// Launch wrappers of the device kernels (host-callable).
#pragma once

#include "common.h"

#include <vector>

// Fine operator data on the device in compute precision T.
//   links  [4][9][V] cplx<T>: U_mu(x), row-major 3x3, with the antiperiodic
//          time sign folded into the links that cross the time boundary
//   clover [72][V] T: two chiral 6x6 Hermitian blocks (A + (m0+4)), each packed
//          as 6 real diagonal entries followed by 15 complex upper entries
template <typename T>
struct FineOp {
  FineGeom g;
  const cplx<T>* links = nullptr;
  const T* clover = nullptr;
};

// Sigma-tensor table: for each plane (mu<nu, 6 planes) and chirality s, the
// 2x2 block of c_sw (i/2) sigma_{mu nu} acting on the two spins of chirality s.
struct CloverCoef {
  double re[6][2][2][2];
  double im[6][2][2][2];
  double diag;   // m0 + 4
};

// ---- conversion (K12) and clover build (K2)
void launch_convert_links(const FineGeom& g, const cplx<double>* canon, cplx<double>* out64,
                          cplx<float>* out32, int antiperiodic, hipStream_t st);
template <typename T>
void launch_spinor_to_internal(const FineGeom& g, const cplx<double>* canon, cplx<T>* out, int nrhs, hipStream_t st);
template <typename T>
void launch_spinor_to_canonical(const FineGeom& g, const cplx<T>* in, cplx<double>* canon, int nrhs, hipStream_t st);
void launch_clover_build(const FineGeom& g, const cplx<double>* links64, const CloverCoef& cc,
                         double* clov64, float* clov32, hipStream_t st);

// ---- fine stencil (K1): out_r = D(mu_r) in_r
template <typename T>
void launch_dslash(const FineOp<T>& op, const cplx<T>* in, cplx<T>* out, int nrhs,
                   const double* mu_dev, hipStream_t st);
// ---- even-odd reduction: out_r = D_hat(mu_r) in_r on the even sites (odd
// outputs 0; odd inputs ignored), tmp: scratch field of the same size
template <typename T>
void launch_schur(const FineOp<T>& op, const cplx<T>* in, cplx<T>* tmp, cplx<T>* out, int nrhs, const double* mu_dev,
                  hipStream_t st);
// zero the sites of one parity (x + y + z + t even: 0, odd: 1)
template <typename T>
void launch_zero_parity(const FineGeom& g, cplx<T>* v, int nrhs, int parity, hipStream_t st);
// out_r = Gamma5 in_r (any level: d dof per site, sites*d elements, SoA fine or AoS coarse)
template <typename T>
void launch_gamma5_fine(const FineGeom& g, const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st);

// ---- fine SAP (K3): one colour's block solves, z updated in place
// epsbar != 0 (FP32, nrhs = 2): the doublet's coupled block operator
template <typename T>
void launch_sap_fine(const FineOp<T>& op, const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu_dev,
                     const int* block_list, int nblk, int mr_steps, hipStream_t st, double epsbar = 0.0);

// the same with two right-hand sides per workgroup (2 x bvol threads);
// lds_bytes: both MR vectors and the reduction slots; n8: blocks rounded up
// to 8; epsbar != 0: the pair is a doublet's two flavours (nrhs = 2) and the
// block operator carries the flavour coupling -epsbar
void launch_sap_fine_pair(const FineOp<float>& op, const cplx<float>* eta, cplx<float>* z, int nrhs,
                          const double* mu_dev, const int* block_list, int nblk, int mr_steps, size_t lds_bytes,
                          unsigned n8, hipStream_t st, double epsbar = 0.0);

// ---- BLAS-1 and Krylov scalars (K9, K10)
struct Reducer {
  double* partial = nullptr;   // [nrhs][nvec][NB] complex as 2 doubles
  int nb_max = 0;
};
int reduce_blocks(long n);
template <typename T>
void launch_multidot(const cplx<T>* V, long vstride, int nvec, const cplx<T>* w, long n, int nrhs,
                     double* partial, int NB, const int* active, hipStream_t st);
// mask (may be null): outputs of right-hand sides with mask[r] == 0 are left as they are
void launch_finalize(const double* partial, int nout, int nvec, int NB, double* out, int ostride, hipStream_t st,
                     const int* mask = nullptr);
template <typename T>
void launch_norm2(const cplx<T>* w, long n, int nrhs, double* partial, int NB, const int* active, hipStream_t st);
void launch_finalize_real(const double* partial, int nout, int NB, double* out, hipStream_t st);
// w_r -= sum_i coef[r][i] V_i,r   (coef complex double [nrhs][cstride])
template <typename T>
void launch_multiaxpy(cplx<T>* w, const cplx<T>* V, long vstride, int nvec, const double* coef, int cstride,
                      long n, int nrhs, double sign, const int* active, hipStream_t st);
// y_r = s_r * x_r with s_r real from device (sidx: stride in s)
template <typename T>
void launch_scale_dev(const cplx<T>* x, cplx<T>* y, const double* s, long n, int nrhs, const int* active,
                      hipStream_t st);
template <typename Tin, typename Tout>
void launch_convert(const cplx<Tin>* x, cplx<Tout>* y, long count, hipStream_t st);
template <typename T>
void launch_axpby(const cplx<T>* x, cplx<T>* y, double a, double b, long count, hipStream_t st);
// y = x - y  (per element)
template <typename T>
void launch_xmy(const cplx<T>* x, cplx<T>* y, long count, hipStream_t st);
// y(fp64) += x(T)
template <typename T>
void launch_add_to64(const cplx<T>* x, cplx<double>* y, long count, hipStream_t st);
// doublet flavour coupling: x, y hold two flavours of n elements back to
// back; y_f += a x_{1-f} (x and y distinct)
template <typename T>
void launch_flavour_couple(const cplx<T>* x, cplx<T>* y, double a, long n, hipStream_t st);
// out = a + c b (complex c), n complex doubles; out may alias a
void launch_lincomb(const cplx<double>* a, const cplx<double>* b, cplx<double>* out, double cre, double cim, long n,
                    hipStream_t st);
// streaming copy of bytes (a multiple of 16)
void launch_copy16(const void* in, void* out, size_t bytes, hipStream_t st);
void launch_fill_zero(void* p, size_t bytes, hipStream_t st);
// dst[i] = vals[i] for i < n, the values carried in the launch arguments:
// the host array need not outlive the call (an asynchronous copy from it
// would read it only when the stream reaches the copy)
void launch_set_doubles(double* dst, const double* vals, int n, hipStream_t st);
// workgroups of 256 for an elementwise launch over count elements: one
// element per thread up to 2^28 elements, beyond that the kernels stride
// by the grid (a launch holds fewer than 2^32 threads)
inline unsigned grid1d(size_t count) {
  const size_t g = (count + 255) / 256;
  return (unsigned)(g == 0 ? 1 : (g > ((size_t)1 << 20) ? ((size_t)1 << 20) : g));
}

struct KrylovDev {
  int m = 0, nrhs = 0;
  double* H = nullptr;       // [nrhs][m+1][m] complex
  double* cs = nullptr;      // [nrhs][m] complex
  double* sn = nullptr;      // [nrhs][m] complex
  double* g = nullptr;       // [nrhs][m+1] complex
  double* c1 = nullptr;      // [nrhs][m+1] complex (first CGS pass)
  double* c2 = nullptr;      // [nrhs][m+1] complex (second CGS pass)
  double* nrm = nullptr;     // [nrhs] real (norms)
  double* inv = nullptr;     // [nrhs] real
  double* beta0 = nullptr;   // [nrhs] real
  double* tol = nullptr;     // [nrhs] real: absolute target
  double* y = nullptr;       // [nrhs][m] complex
  int* active = nullptr;     // [nrhs]
  int* kdone = nullptr;      // [nrhs]
  int* status = nullptr;     // [nrhs]: 0 running, 1 converged, 2 breakdown/NaN
  int* reorth = nullptr;     // [nrhs]: second Gram-Schmidt pass needed this step
};
// start of a cycle: nrm holds ||r||, sets beta0, g, active, inv
void launch_krylov_start(const KrylovDev& k, double reltol, const double* abstol, int nrhs, hipStream_t st);
// after the first classical Gram-Schmidt pass of step j (c1 holds the j + 1
// coefficients and, at j + 1, |w|^2 before the pass): reorth[r] = 1 where the
// pass cancelled more than the factor eta2 of |w|^2 (|w'|^2 = |w|^2 - sum |c1|^2
// < eta2 |w|^2), else c2 is zeroed and the second pass is skipped
void launch_cgs_decide(const KrylovDev& k, int j, int nrhs, double eta2, hipStream_t st);
// iteration j: c1 + c2 -> H column, nrm -> h_{j+1,j}; Givens; convergence
void launch_krylov_step(const KrylovDev& k, int j, int nrhs, hipStream_t st);
// triangular solve for y (uses kdone)
void launch_krylov_solve_y(const KrylovDev& k, int nrhs, hipStream_t st);
// x_r += sum_{i<kdone_r} y_i Z_i
template <typename T>
void launch_krylov_update(cplx<T>* x, const cplx<T>* Z, long zstride, const KrylovDev& k, long n, int nrhs,
                          hipStream_t st);

// ---- multigrid transfer, coarse operator, setup (K4-K8, K11)
// P storage: N_v fields of the finer level in storage precision S; column
// (s, i) of P is field i restricted to the chirality-s half of the dofs and
// to one aggregate.  Coarse fields: [nrhs][Vc][d] cplx<T>, dof index s*N_v + i.
// D_c storage: [Vc][9][d][d] column-major blocks (j slow, i fast); block 0 is
// the self block, 1+2mu couples to y+mu, 2+2mu to y-mu.
template <typename T, typename S>
void launch_restrict_fine(const FineGeom& g, const typename Store<S>::pair* P, int nv, const cplx<T>* in,
                          cplx<T>* out, int nrhs, hipStream_t st);
template <typename T, typename S>
void launch_prolong_fine(const FineGeom& g, const typename Store<S>::pair* P, int nv, const cplx<T>* in,
                         cplx<T>* out, int nrhs, hipStream_t st);
template <typename T, typename S>
void launch_restrict_coarse(const CoarseGeom& g, int d, const int agg[4], const typename Store<S>::pair* P, int nv,
                            const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st);
template <typename T, typename S>
void launch_prolong_coarse(const CoarseGeom& g, int d, const int agg[4], const typename Store<S>::pair* P, int nv,
                           const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st);
template <typename T, typename S>
void launch_coarse_apply(const CoarseGeom& g, int d, const typename Store<S>::pair* Dc, const cplx<T>* in,
                         cplx<T>* out, int nrhs, const double* mu_dev, hipStream_t st);
template <typename T, typename S>
void launch_sap_coarse(const CoarseGeom& g, int d, const int blk[4], const typename Store<S>::pair* Dc,
                       const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu_dev, const int* blist, int nblk,
                       int mr_steps, hipStream_t st);
template <typename T>
void launch_gamma5_coarse(long V, int d, const cplx<T>* in, cplx<T>* out, int nrhs, hipStream_t st);
// block Gram-Schmidt (FP64): tv (T) -> P64 scratch and P (S)
bool gs_fine_needs_fp64_copy(int nv);
template <typename T, typename S>
void launch_gs_fine(const FineGeom& g, const cplx<T>* tv, int nv, cplx<double>* P64, typename Store<S>::pair* P,
                    hipStream_t st);
template <typename T, typename S>
void launch_gs_coarse(const CoarseGeom& g, int d, const int agg[4], const cplx<T>* tv, int nv, cplx<double>* P64,
                      typename Store<S>::pair* P, hipStream_t st);
// Galerkin D_c = P^dag D P (without the twisted-mass term).  zws: workspace
// of zws_elems complex values, at least galerkin_ws_per_column(g); larger
// workspaces process more columns per pass (up to 16).
size_t galerkin_ws_per_column(const FineGeom& g);
template <typename T, typename S>
void launch_galerkin_fine(const FineOp<T>& op, const typename Store<S>::pair* P, int nv,
                          typename Store<S>::pair* Dc, cplx<T>* zws, size_t zws_elems, hipStream_t st);
template <typename T, typename S>
void launch_galerkin_coarse(const CoarseGeom& g, int d, const int agg[4], const typename Store<S>::pair* Dc1,
                            const typename Store<S>::pair* P, int nv, typename Store<S>::pair* Dc2, hipStream_t st);
// complex Gaussian noise, E|z|^2 = 1, counter-based (seed, index)
template <typename T>
void launch_random(cplx<T>* out, long count, unsigned long long seed, hipStream_t st);
// D_c(mu_r) with one coarse site per workgroup (false: shape not covered)
template <typename T, typename S>
bool launch_coarse_apply_site(const CoarseGeom& g, int d, const typename Store<S>::pair* Dc, const cplx<T>* in,
                              cplx<T>* out, int nrhs, const double* mu_dev, hipStream_t st);
// Coarse-level SAP with fused MR launches, and the persistent coarsest
// GMRES (false: shape not covered, the caller uses the generic kernels)
template <typename T, typename S>
bool launch_sap_coarse_fused(const CoarseGeom& g, int d, const int blk[4], const typename Store<S>::pair* Dc,
                             const cplx<T>* eta, cplx<T>* z, int nrhs, const double* mu_dev, const int* bl0, int n0,
                             const int* bl1, int n1, int sweeps, int mr_steps, cplx<T>* const rho[2],
                             cplx<T>* const q[2], double* const part[2], long part_cap, hipStream_t st);
int coarsest_groups(long nsites);
size_t coarsest_ws_doubles(int nrhs, int m, int G);
size_t coarsest_ws_ints(int nrhs);
template <typename T, typename S>
bool launch_coarsest_gmres(const CoarseGeom& g, int d, const typename Store<S>::pair* Dc, const cplx<T>* b, cplx<T>* x,
                           int nrhs, const double* mu_dev, int m, double reltol, cplx<T>* Vbasis, cplx<T>* w,
                           double* dws, size_t dws_cap, int* iws, size_t iws_cap, hipStream_t st);
// storage conversions for the debug/export hooks
template <typename S>
void launch_store_to64(const typename Store<S>::pair* in, cplx<double>* out, long count, hipStream_t st);
template <typename S>
void launch_store_from64(const cplx<double>* in, typename Store<S>::pair* out, long count, hipStream_t st);
// fine field SoA [nrhs][12][V] <-> AoS [nrhs][V][12] lexicographic-free copy helpers are not needed:
// per-level exports go through launch_spinor_to_canonical (fine) or plain copies (coarse).

// ------------------------------------------------------------------ kernel variant table
// Families with more than one correct kernel per shape (same numbering as
// TMAMG_TUNE_* in the public header).  Keys are (a, b, c) per family:
//   TUNE_COARSE_APPLY (d, coarse sites, nrhs): 0 vector ALU, 1 matrix cores
//   TUNE_SAP1         (d, coarse sites, nrhs): 0 vector ALU, 1 matrix cores,
//                     2 matrix cores with a register budget for four workgroups per CU,
//                     3 matrix cores, one workgroup per SAP block (blocks of at most 16 sites)
//   TUNE_RESTRICT0 / TUNE_PROLONG0 (nv, fine sites, nrhs): 0 vector ALU, 1 matrix cores
//   TUNE_SAP0         (block sites, fine sites, nrhs): register budget for 0 one, 1 three workgroups per CU;
//                     2: two right-hand sides per workgroup (lane pairs share every link and clover load)
// tune_get returns -1 without an entry; the launcher then applies its own
// rule, and records the variant it ran with tune_used.
enum { TUNE_COARSE_APPLY = 0, TUNE_SAP1, TUNE_RESTRICT0, TUNE_PROLONG0, TUNE_SAP0, TUNE_NFAM };
constexpr int TUNE_MAX_VARIANTS = 4;
inline int tune_variants(int family) { return family == TUNE_SAP1 ? 4 : family == TUNE_SAP0 ? 3 : 2; }
int tune_get(int family, long a, long b, long c);
void tune_put(int family, long a, long b, long c, int variant, const double* ms, int nms);
void tune_used(int family, int variant);
int tune_last_used(int family);
void tune_clear();
int tune_entries();
bool tune_save(const char* path, const char* device);
int tune_load(const char* path);
const char* tune_family_name(int family);
