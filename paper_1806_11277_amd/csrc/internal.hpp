// Host-side declarations shared by the kernel files and the C ABI implementation.
#pragma once

#include "common.hpp"

#define EHH_KMAXV 17   // restart length + 1

namespace ehh {

// Operator of one multigrid level in precision T: matrix-free on level 0 of a
// (sub)domain, Galerkin stencils on the coarser levels.
// Row coefficients of the 2D half-sweep stored in its lane order (one set per
// colour): term j of lane i at [j * lanes + i], real parts of all terms,
// imaginary parts of the u-u terms; null where a level builds its rows in the
// kernel.  Columns are computed from the row's position.
template <typename T> struct StoredPlan {
    const T* re[2] = {nullptr, nullptr};
    const T* im[2] = {nullptr, nullptr};
    int64_t lanes = 0;
    // rows of y = A x in row order (term j of row t at [j * N + t])
    const T* rre = nullptr;
    const T* rim = nullptr;
    // complex64 cycle with FP16 rows: the pointers above hold FP16 values, the
    // coefficients divided by scale (a power of two)
    bool half = false;
    float scale = 1.0f;
};

template <typename T> struct LevelDesc {
    Geo g;
    bool fine;
    FineCoef<T> f;
    StCoef<T> s;
    StoredPlan<T> sp;
    // source groups per launch chosen by the autotuner for the level's half-sweeps
    // and residuals (0: the launchers' own heuristic); launch shapes only, the
    // arithmetic of every source is the same for any value
    int tune_relax = 0, tune_apply = 0;
};

// Vanka damping of one level: u for the displacement rows of a cell block, p for
// its pressure row (the component-dependent damping W = diag(w_u, .., w_p) of
// the damped block update in section 5.2; u == p for the plain damping).
struct Damp {
    double u, p;
};

// ---- levels.hip
template <typename T>
hipError_t launch_apply(const LevelDesc<T>& L, const T* x, const T* b, T* y, int nrhs, hipStream_t s);
// y = A x on a finest level (2D or 3D, one-thread-per-cell kernels) with x in
// FP32; apply_x32_supported tells whether the level qualifies.
bool apply_x32_supported(const LevelDesc<double>& L);
hipError_t launch_apply_x32(const LevelDesc<double>& L, const float* x, double* y, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_relax(const LevelDesc<T>& L, int colour, Damp w, int econ, const T* b, const T* ein,
                        T* eout, int nrhs, hipStream_t s);
// Colour-1 half-sweep of a finest 2D level with an FP64 e_out (*done = false
// where no kernel serves it: the caller then converts after the cycle).
hipError_t launch_relax_to64(const LevelDesc<float>& L, Damp w, int econ, const float* b, const float* ein,
                             double* eout, int nrhs, hipStream_t s, bool* done);
// First half-sweep (colour 0) of a visit from zero with the restriction fused:
// b = P^T rf (rf on the finer grid gf) is formed, written to b, and relaxed.
template <typename T>
bool relax_restrict_supported(const LevelDesc<T>& L, const Geo& gf, int nrhs);
template <typename T>
hipError_t launch_relax_restrict(const LevelDesc<T>& L, Damp w, int econ, const Geo& gf, const T* rf, T* b,
                                 T* eout, int nrhs, hipStream_t s);
// Lanes (padded) of one colour's stored plans on a level, and the builder.
int64_t stored_plan_lanes(const Geo& g);
bool stored_plan_wanted(const Geo& g, bool fine);
int stored_terms(int dim);        // real parts per stored row
int stored_imag_terms(int dim);   // imaginary parts per stored row (the u-u terms)
template <typename T>
hipError_t launch_build_plans(const LevelDesc<T>& L, int colour, T* re, T* im, hipStream_t s);
template <typename T>
hipError_t launch_build_row_plans(const LevelDesc<T>& L, T* re, T* im, hipStream_t s);
// rc = P^T (b - A e) in one launch from a 2D level with stored rows (vectors of
// nrhs sources back to back); *done = false (nothing launched) elsewhere.
template <typename T>
hipError_t launch_residual_restrict(const LevelDesc<T>& L, const Geo& gc, const T* e, const T* b, T* rc, int nrhs,
                                    hipStream_t s, bool* done);
// FP16 copies of stored rows: *out = max over x of |x| as float bits (out
// zeroed by the caller); y = x * inv_scale rounded to FP16.
hipError_t launch_absmax_bits(const float* x, int64_t n, unsigned* out, hipStream_t s);
hipError_t launch_to_half(const float* x, void* y, int64_t n, float inv_scale, hipStream_t s);
template <typename T>
hipError_t launch_restrict(const Geo& gf, const Geo& gc, const T* rf, T* rc, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_prolong(const Geo& gf, const Geo& gc, const T* ec, T* ef, int nrhs, hipStream_t s);

// ---- setup.hip
// Sums of mu and rho and the number of non-physical cells (non-finite values,
// rho <= 0, mu < 0, lambda + mu <= 0); out[0..2] on the device.
hipError_t launch_media_check(const double* lam, const double* mu, const double* rho, const double* gam,
                              int64_t ncell, double* partial, int nblocks, double* out, hipStream_t s);
int media_check_blocks(int64_t ncell);

struct FineCoefParams {
    int dim;
    int n_glob[3];
    int n_loc[3];
    int origin[3];       // global cell of local cell 0
    int pad_lo[3], pad_hi[3];
    int abl[3];
    double abl_max;
    double gam0;         // atten0 / omega
    double inv_omega;    // 1 / omega (for the physical attenuation)
    double mu_bar, rho_bar;
};
// mu, dinv, rho, gam planes (4 * ncell_loc doubles) of a (sub)domain level 0.
hipError_t launch_fine_coef(const FineCoefParams& p, const double* lam, const double* mu, const double* rho,
                            const double* gam_phys, double* out, hipStream_t s);
// Level-0 shifted operator written in the stencil format of the coarse levels.
hipError_t launch_materialise(const Geo& g, const FineCoef<double>& c, double* st, hipStream_t s);
// Galerkin product P^T A P: stencil of grid gf -> stencil of grid gc.
hipError_t launch_galerkin(const Geo& gf, const double* stf, const Geo& gc, double* stc, hipStream_t s);
// Dense row-major complex (re, im interleaved) matrix of a stencil-format level.
hipError_t launch_dense_assemble(const Geo& g, const double* st, double* dense, hipStream_t s);
// In-place blocked Gauss-Jordan inversion of a dense n x n complex matrix,
// pivoting inside 64 x 64 diagonal blocks: leaves (Pi A)^{-1}, with the row
// interchanges in piv[0..n) (row k swapped with row piv[k], in order) and
// *flag = 1 on a zero pivot.
hipError_t launch_dense_invert(double* dense, int64_t n, int* piv, int* flag, hipStream_t s);
// out[i][j] = X[i][qinv[j]] (n x n complex, out-of-place).
hipError_t launch_permute_columns(const double* X, double* out, int64_t n, const int* qinv, hipStream_t s);
// e = inv r for a batch of right-hand sides (FP64 accumulation).
template <typename T>
hipError_t launch_coarse_apply(const double* inv, const double* sym, int64_t n, const T* r, T* e, int nrhs,
                               double* ws, hipStream_t s);
// Scratch array of the coarsest solve that allocates nothing: kNoallocScratchDoubles
// FP64 values per device (32 MiB).  noalloc_scratch_init takes the address of
// device dev's copy (dev must be current) once; noalloc_scratch returns it
// (null before the first init on that device).
constexpr int64_t kNoallocScratchDoubles = int64_t(1) << 22;
constexpr int kMaxDevices = 64;
hipError_t noalloc_scratch_init(int dev);
double* noalloc_scratch(int dev);
// Packed lower tiles of the (symmetric) inverse, used by launch_coarse_apply.
int64_t sym_tiles(int64_t n);
hipError_t launch_pack_sym(const double* inv, int64_t n, double* sym, hipStream_t s);
// Column segments of the coarse apply and the FP64 workspace they need (0: none).
int coarse_ksplit(int64_t n, int nrhs);
size_t coarse_ws_doubles(int64_t n, int nrhs);
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);   // bytes multiple of 4
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t s);

// ---- dd.hip
struct SubMap {
    int dim;
    int origin[3];
    int lo[3], hi[3];
    const int* cnt_cell[3];   // per axis: subdomains covering cell c (global)
    const int* cnt_face[3];   // per axis: subdomains owning face position f (global)
};
template <typename T>
hipError_t launch_dd_gather(const Geo& gg, const Geo& gl, const SubMap& m, const double* v, T* out, int nrhs,
                            hipStream_t s);
template <typename T>
hipError_t launch_dd_gather_res(const Geo& gg, const Geo& gl, const SubMap& m, const FineCoef<double>& A,
                                const double* v, const double* z, T* out, int nrhs, hipStream_t s);
template <typename T>
hipError_t launch_dd_scatter(const Geo& gg, const Geo& gl, const SubMap& m, const T* e, double* z, int nrhs,
                             int weighted, hipStream_t s);

// DD as the coarsest-grid solver: device index arrays of the boxes (subdomains)
// of a coarsest level, local unknowns numbered box after box.
struct BoxMap {
    const int* map;        // coarsest unknown of each local unknown
    const int* bsub;       // box of each local unknown
    const int64_t* bbase;  // first local unknown of each box
    const int* bn;         // unknowns of each box
};
// Stencil of the box [lo, lo + gb.n) of the coarsest grid gc, on the box's grid.
hipError_t launch_box_stencil(const Geo& gc, const double* stc, const Geo& gb, double* stb, const int* lo,
                              hipStream_t s);
// loc <- src on the local unknowns [j0, j1); z += (wgt or 1) loc there.
hipError_t launch_box_gather(const BoxMap& m, int64_t j0, int64_t j1, const double* src, int64_t Nc, double* loc,
                             int nrhs, hipStream_t s);
hipError_t launch_box_scatter(const BoxMap& m, int64_t j0, int64_t j1, const double* loc, const double* wgt,
                              int64_t Nc, double* z, int nrhs, hipStream_t s);

// ---- krylov.hip (FP64, vectors of 2N reals per right-hand side)
int krylov_blocks(int64_t n2);
// nrm2[r] = |x(r)|^2
hipError_t launch_norm2(const double* x, int64_t N, int nrhs, double* partial, double* nrm2, hipStream_t s);
// out(r) = x(r) * scale[r] (scale real; mode 1: 1/sqrt(scale[r])); out32, if
// not null, receives an FP32 copy.
hipError_t launch_scale(const double* x, double* out, int64_t N, int nrhs, const double* scale, int mode,
                        hipStream_t s, float* out32 = nullptr);
// One Arnoldi orthogonalisation for every right-hand side (nv <= m): w(r)
// against V_0(r) .. V_{nv-1}(r) by classical Gram-Schmidt, h1 = V^H w; where
// the pass kept less than 0.1 of |w| (or always, force_two) a second pass
// h2 = V^H w' follows, h2 = 0 elsewhere.  The normalised result goes to
// vnext(r) (and v32(r), if given) and its squared norm to nrm2[r]; w is
// scratch.  h1, h2: (m + 1) complex entries per source (slot m is scratch:
// |w|^2 in h1, the one-pass flag in h2); partial: krylov_blocks * nrhs *
// (m + 1) * 2 doubles.
hipError_t launch_orthogonalise(const double* V, int nv, double* w, int64_t N, int nrhs, double* partial,
                                double* h1, double* h2, int m, double* nrm2, double* vnext, float* v32,
                                bool force_two, hipStream_t s);
// Givens update of column j of every right-hand side's Hessenberg matrix:
// entries hcol + hcol2 (i <= j) and sqrt(nrm2[r]) below the diagonal.
hipError_t launch_givens(double* H, double* cs, double* g, const double* hcol, const double* hcol2,
                         const double* nrm2, int j, int m, int nrhs, const int* active, double* est,
                         const double* bnorm, hipStream_t s);
// y = R^{-1} g (columns ncols[r]); x(r) += sum_i y_i Z_i(r)
hipError_t launch_update_x(const double* H, const double* g, const double* Z, double* x, int64_t N, int nrhs,
                           int m, const int* ncols, double* y, hipStream_t s);
hipError_t launch_update_x(const double* H, const double* g, const float* Z, double* x, int64_t N, int nrhs,
                           int m, const int* ncols, double* y, hipStream_t s);   // Z in FP32

hipError_t launch_axpby(const double* x, const double* y, double* out, int64_t n, double a, double b,
                        hipStream_t s);

// ---- gradient.hip
// y = conj(x) for nrhs vectors of the global layout (x == y allowed).
hipError_t launch_conj(const double* x, double* y, int64_t N, int nrhs, hipStream_t s);
// Per cell: dL/d{lambda, mu, rho} = -Re sum_r y_r^H (dA/dm) x_r in SI units
// (fine = mu, dinv, rho, gamma planes of the global operator).
hipError_t launch_media_gradient(const Geo& g, const double* fine, double om2, const double* y, const double* x,
                                 int nrhs, double mu_bar, double rho_bar, double* gl, double* gm, double* gr,
                                 int accumulate, hipStream_t s);

}  // namespace ehh
