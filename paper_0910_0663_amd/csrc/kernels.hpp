// Launchers of the HIP kernels (gfx950).  All take the stream to run on and
// return the launch status; none synchronizes.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <utility>

#include "tiles.hpp"

namespace vtm {

// Raises kern's dynamic LDS limit on the current device to at least lds bytes
// (launches above 64 KiB need it).  A (kernel, device) pair is raised only when a
// larger size comes, under a lock, so handles on different host threads may
// launch the same kernel together.
inline hipError_t raise_lds_limit(const void* kern, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, size_t> raised;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    size_t& cur = raised[{kern, dev}];
    if (lds <= cur) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e == hipSuccess) cur = lds;
    return e;
}

// Largest sub-circuit whose local matrix is factored entirely in LDS.
constexpr int kLdsSetupMax = 80;

// Coupled lines: the outgoing wave of port p is sum_k val[k] x_node(col[k]) +
// gamma_p a_p over k in [row[p], row[p + 1]) (B = 2 W over the ports of p's
// sub-circuit).  row == nullptr: diagonal lines, B = diag(beta).
template <typename T>
struct Coupling {
    const int32_t* row = nullptr;
    const int32_t* col = nullptr;
    const T* val = nullptr;
};

struct PortArrays {
    const int32_t* off;    // [S + 1]
    const int32_t* node;   // local node of each port
    const int32_t* slot;   // rank among the ports of its node
    const int32_t* twin;   // port receiving this port's outgoing wave
    int max_slot;
};

// ---- setup ----------------------------------------------------------------
// Forms K_s = A_ss + diag(dmod) (the cut branch g replaced by the port
// conductance G at every port node) for every sub-circuit and writes K_s^-1 in
// the column-group layout of layout.hpp into out + kofs[s].  Sub-circuits with
// ns <= kLdsSetupMax are inverted in LDS; larger ones are assembled into
// scratch64 (FP64, same offsets, must be non-null then) and inverted there by a
// blocked Gauss-Jordan elimination with partial pivoting, whose panels use
// panel (setup_panel_doubles(n, max_ns) doubles) and ipiv (n ints), both
// non-null then.  flag bit 0 = singular.
int64_t setup_panel_doubles(int64_t n, int max_ns);

template <typename TO>
hipError_t launch_setup(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs,
                        const int32_t* rowptr, const int32_t* col, const double* val,
                        const double* dmod, TO* out, double* scratch64, double* panel, int32_t* ipiv,
                        int* flag, hipStream_t st);

// Same matrices, written as zero-padded MFMA operand tiles (tiles.hpp) of T
// (BF16 or FP64) at out + mofs[s]; every sub-circuit passes through FP64
// column-major scratch64 (kofs offsets, required).  out_t (nullable) receives
// the transposed inverses K_s^-T in the same layout (the adjoint's operator).
template <typename T>
hipError_t launch_setup_tiles(int S, int max_ns, const int32_t* sub_off, const int64_t* kofs,
                              const int64_t* mofs, const int32_t* rowptr, const int32_t* col,
                              const double* val, const double* dmod, T* out, double* scratch64, double* panel,
                              int32_t* ipiv, int* flag, hipStream_t st, T* out_t = nullptr);

// ---- sweep ----------------------------------------------------------------
// One VTM sweep for every sub-circuit (one workgroup each, per block of up to 8
// right-hand sides): right-hand side b + c * a at the port nodes,
// x = K^-1 rhs (K^-T when adjoint), then the outgoing wave beta * x + gamma * a
// sent to the twin port in a_next.  Vectors are [rows][nrhs] (right-hand side
// fastest).  port_rows: x may be formed on the port nodes only (numbered first
// in each sub-circuit), all the waves need; the single right-hand-side forward
// sweep does so, the others form every row.
template <typename TO, typename TV>
hipError_t launch_sweep(int S, int max_ns, int nrhs, const TO* K, const int64_t* kofs,
                        const int32_t* sub_off, PortArrays ports, const TV* pc, const TV* pbeta,
                        const TV* pgamma, const TV* b, const TV* a_cur, TV* a_next, TV* x,
                        bool adjoint, size_t lds_limit, hipStream_t st, bool port_rows = false);

// Batched sweep on MFMA (mfma.hip) with the inverses in tile layout: per
// sub-circuit X = Kinv [b + c a] for blocks of up to 64 right-hand sides, then
// the outgoing waves.  variant: 0 gives each wavefront 3 row tiles per pass, 1
// gives it 5; rc_req: right-hand sides per workgroup (multiple of 16; 0 =
// widest that fits lds_limit).  write_x = false stores x on port rows only (enough
// for the waves; pass true on the last sweep before a residual check); port_rows
// forms x only in the row tiles that hold port nodes (numbered first in each
// sub-circuit).  The BF16 form reads b in BF16.  The adjoint passes the tiles of
// K^-T as K.
template <typename T>
hipError_t launch_sweep_mfma(int S, int max_ns, int max_ports, int nrhs, int variant, int rc_req,
                             size_t lds_limit, const T* K, const int64_t* mofs, const int32_t* sub_off,
                             PortArrays ports, const typename MfmaTypes<T>::TV* pc,
                             const typename MfmaTypes<T>::TV* pbeta, const typename MfmaTypes<T>::TV* pgamma,
                             const typename MfmaTypes<T>::TB* b, const typename MfmaTypes<T>::TV* a_cur,
                             typename MfmaTypes<T>::TV* a_next, typename MfmaTypes<T>::TV* x, bool write_x,
                             hipStream_t st, bool port_rows = false);
// Batched port-to-port sweep: a_next[twin(p)][r] = h[p][r] + (M_s a_cur)_p[r] per
// sub-circuit, M_s (q x q) in A-tile order at Mop + qmofs[s] (padded to
// roundup(q, 32)); variant bit 0 as above (5 row tiles per pass, else 3), bit 1
// = 8 wavefronts per workgroup (else 4); rc_req as above.
template <typename T>
hipError_t launch_sweep_mfma_pp(int S, int max_ports, int nrhs, int variant, int rc_req, size_t lds_limit,
                                const T* Mop, const int64_t* qmofs, const int32_t* port_off,
                                const int32_t* port_twin, const typename MfmaTypes<T>::TV* h,
                                const typename MfmaTypes<T>::TV* a_cur, typename MfmaTypes<T>::TV* a_next,
                                int reverse, hipStream_t st);
// M_s = diag(beta) Kinv[P, P] diag(c) + diag(gamma) in A-tile order from the FP64
// column-major inverses at Kinv + kofs[s] (coefficients FP64, rounded to T once).
template <typename T>
hipError_t launch_port_matrix_tiles(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* port_off,
                                    const int32_t* port_node, const double* pc, const double* pbeta,
                                    const double* pgamma, const double* Kinv, const int64_t* qmofs, T* out,
                                    hipStream_t st, Coupling<double> B = {});

// ---- port-to-port form (ports.hip) -------------------------------------------
// M_s = diag(beta) K^-1[i(P), i(P)] diag(c) + diag(gamma) for every sub-circuit,
// from the stored inverses (column-group layout), into M + pofs[s] (same layout,
// n = q_s).  Coefficients in FP64.
template <typename TO>
hipError_t launch_port_matrix(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* port_off,
                              const int32_t* port_node, const double* pc, const double* pbeta,
                              const double* pgamma, const TO* K, const int64_t* pofs, TO* M, hipStream_t st,
                              Coupling<double> B = {});
// h_p = beta_p x_i(p), or (B x)_p with coupled lines (x renumbered)
template <typename TV>
hipError_t launch_port_h(int S, int nrhs, const int32_t* sub_off, const int32_t* port_off, const int32_t* port_node,
                         const TV* pbeta, const TV* x, TV* h, hipStream_t st, Coupling<TV> B = {});
// Coupled lines, after a full sweep: a_next[twin(p)] = sum_m B_pm x_row(m) +
// gamma_p a_cur[p] for every port and right-hand side (replaces the diagonal
// waves the sweep wrote; x and waves [rows][nrhs]).
template <typename TV>
hipError_t launch_wave_coupled(int n_ports, int nrhs, Coupling<TV> B, const int32_t* port_row, const TV* pgamma,
                               const int32_t* port_twin, const TV* x, const TV* a_cur, TV* a_next, hipStream_t st);
// a_next[twin(p)] = h_p + (M_s a_cur)_p for every port (one right-hand side)
template <typename TO, typename TV>
hipError_t launch_sweep_pp(int S, int max_q, const TO* M, const int64_t* pofs, const int32_t* port_off,
                           const int32_t* port_twin, const TV* h, const TV* a_cur, TV* a_next, hipStream_t st);

// Port-node form for any A: K^-1[N, N] over a sub-circuit's k port nodes in the
// column-group layout (n = k) at Sn + nofs[s] (transpose: K^-T[N, N], for the
// adjoint of an unsymmetric A) ...
template <typename TO>
hipError_t launch_port_node_dense(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* pn_off,
                                  const int32_t* pn_node, const TO* K, const int64_t* nofs, TO* Sn, bool transpose,
                                  hipStream_t st);
// ... and its sweep: t_n = sum_{p at n} c_p a_p, z = K^-1[N, N] t,
// a_next[twin(p)] = beta_p z_n(p) + gamma_p a_p + h_p (LDS 2 max_npn values +
// 4 max_ports bytes, at most 64 KiB, else hipErrorInvalidValue).
template <typename TO, typename TV>
hipError_t launch_sweep_ppn(int S, int max_npn, int max_ports, const TO* Sn, const int64_t* nofs,
                            const int32_t* pn_off, const int32_t* pn_pfirst, const int32_t* port_off,
                            const int32_t* port_twin, const TV* pc, const TV* pbeta, const TV* pgamma, const TV* h,
                            const TV* a_cur, TV* a_next, hipStream_t st);

// Symmetric A: upper triangle of S = K^-1[port nodes, port nodes] per
// sub-circuit as row-interleaved pairs of diagonals (pair m from 2m (k - m + 1),
// k port nodes; pads zero), block start 16-byte aligned, at Sp + sofs[s] ...
template <typename TO>
hipError_t launch_port_node_matrix(int S, const int32_t* sub_off, const int64_t* kofs, const int32_t* pn_off,
                                   const int32_t* pn_node, const TO* K, const int64_t* sofs, TO* Sp,
                                   hipStream_t st);
// ... and the port-to-port sweep on it: t_n = sum_{p at n} c_p a_p, z = S t,
// a_next[twin(p)] = 2 W_p c_p z_n(p) + (1 - 2 c_p) a_p + h_p (pW null: W for
// every port).  Needs at most 64 port nodes and 64 ports per sub-circuit (else
// hipErrorInvalidValue); two sub-circuits share a wavefront when both maxima
// are at most 32.  reverse != 0 walks the sub-circuits in reverse order (the
// solver alternates it, so each sweep starts on the operators the previous one
// read last); results do not depend on it.
template <typename TO, typename TV>
hipError_t launch_sweep_pps(int S, int max_npn, int max_ports, const TO* Sp, const int64_t* sofs,
                            const int32_t* pn_off, const int32_t* pn_pfirst, const int32_t* port_off,
                            const int32_t* port_twin, const TV* pc, const TV* pW, TV W, const TV* h,
                            const TV* a_cur, TV* a_next, int reverse, hipStream_t st);

// ---- residual -------------------------------------------------------------
// Per right-hand side, the sum of squares of b - A x for the iterate of the
// sweep that read a_cur and wrote a_next ([ports][nrhs]), from port quantities
// alone: norms[2 r] (norms[2 r + 1] = 0).  pn_pfirst[n] .. pn_pfirst[n + 1] are
// the ports of port node n (n < count).  partial: kResidBlocks * nrhs * 2 doubles.
template <typename TV>
hipError_t launch_port_residual(int64_t n_port_nodes, int nrhs, const int32_t* pn_pfirst, const int32_t* twin,
                                const TV* a_cur, const TV* a_next, const double* c, const double* beta,
                                const double* gamma, const double* gd, const double* g, double* partial, double* norms,
                                hipStream_t st);
// r = b - A x in FP64 on the untorn (renumbered) A; per right-hand side
// sums of r^2 and b^2 land in norms[2 * rhs + {0, 1}] (fixed summation order).
// r_out may be null.  partial must hold kResidBlocks * nrhs * 2 doubles.
// Largest number of workgroups of the residual kernels.  They take one per 4,096
// (row, right-hand side) pairs, at least 1,024: with many right-hand sides a
// row's gathers are one wavefront's dependent loads, and more wavefronts hide
// them; small problems keep fewer partial sums.
constexpr int kResidBlocks = 4096;
inline int resid_blocks(int64_t rows, int nrhs) {
    const int64_t b = rows * nrhs / 4096;
    return int(b < 1024 ? 1024 : (b > kResidBlocks ? kResidBlocks : b));
}
// r_out (FP64), r32 (FP32) and r16 (BF16) are optional copies of r = b - A x
template <typename TX>
hipError_t launch_residual(int n, int nrhs, const int32_t* rowptr, const int32_t* col,
                           const double* val, const double* b, const TX* x, double* r_out, float* r32,
                           __bf16* r16, double* partial, double* norms, hipStream_t st);

// ---- vector utilities -------------------------------------------------------
// dst[i][r] = src[r][perm[i]]   (column-major caller layout -> renumbered rows)
// Vertex tearing: out[r][j] = w[r] * in(src[r], j) per plan row r, the input a
// caller's [nrhs][n_in] vector (in_rhs_major) or [n_in][nrhs] ...
hipError_t launch_expand(int rows, int nrhs, int n_in, const int32_t* src, const double* w, const double* in,
                         bool in_rhs_major, double* out, hipStream_t st);
// ... and back: out(i, j) = x[r0[i]][j], or the mean with x[r1[i]][j] when r1[i] >= 0.
template <typename TX>
hipError_t launch_restrict(int n, int nrhs, const int32_t* r0, const int32_t* r1, const TX* x, double* out,
                           bool out_rhs_major, hipStream_t st);
hipError_t launch_gather(int n, int nrhs, const int32_t* perm, const double* src, double* dst,
                         hipStream_t st);
// dst[r][j] = src[iperm[j]][r]
hipError_t launch_scatter(int n, int nrhs, const int32_t* iperm, const double* src, double* dst,
                          hipStream_t st);
template <typename T>
hipError_t launch_fill(int64_t count, T value, T* dst, hipStream_t st);
// dst = (TD) src
template <typename TS, typename TD>
hipError_t launch_convert(int64_t count, const TS* src, TD* dst, hipStream_t st);
// x += (double) d
template <typename TD>
hipError_t launch_add(int64_t count, const TD* d, double* x, hipStream_t st);
// out[r][q] = a[abi2port[q]][r] (get) or a[abi2port[q]][r] = in[r][q] (set)
template <typename TV>
hipError_t launch_waves_io(int64_t np, int nrhs, const int32_t* abi2port, TV* a, double* abi,
                           bool to_abi, hipStream_t st);
// dL_dA[k] = -sum_r lam[r][row[k]] x[r][col[k]] (x, lam: [nrhs][n]; row, col: [nnz], in range)
hipError_t launch_grad_entries(int64_t nnz, int n, int nrhs, const double* x, const double* lam, const int32_t* row,
                               const int32_t* col, double* dL_dA, hipStream_t st);
// dL_dg[e] = -sum_r (lam_i - lam_j)(x_i - x_j)
hipError_t launch_grad(int64_t m, int n, int nrhs, const double* x, const double* lam,
                       const int32_t* ij, double* dL_dg, hipStream_t st);

}  // namespace vtm
