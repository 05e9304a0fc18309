// qt_internal.h -- structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/qtraj.h"

namespace qt {

// Per-trajectory state between segments (and the record of the plain form).
struct TrajState {
    int64_t step;         // steps taken
    int32_t l, c, n_jumps, status;
    int32_t started, done, pad0, pad1;
    double  r, first_r, min_gap, norm;
    double  scl;          // FP32-bulk: the state is scl times the stored values
    double  pad2;
};

// One batch of trajectories that share physics, table and initial state.
struct GroupDesc {
    double  L, dr, dt, mass, alpha, kappa_hat, gamma_hat, r_max;
    double  tau_start;
    int32_t N, do_jumps, max_jumps, init_l, init_color, flags, n_tab, pad0;
    int64_t n_steps, n_traj;
    uint64_t seed, traj_id0, traj_id_stride;
    const double* tau;
    const double* Ttab;
    const void*   kin;        // N kinetic factors (2/N folded in), 16 bytes each:
                              // FP64 complex, or FP32 hi.re hi.im lo.re lo.im
    const double* init_psi;   // 2N doubles (re, im)
    const double* basis;      // 6N doubles
    const double* Tn;         // per-step temperature (plain form only)
    const void*   phase;      // [(2 l + c) N + m]: exp(-i dt/2 V_static), l <= l_tab
    int32_t l_tab, pad1;
    double  init_overlap[6];
    qt_results out;           // device pointers
    void*      st_psi;        // n_traj * N complex (segmented runs), or null
    TrajState* st;            // n_traj records (segmented runs), or null
    qt_results zeroth;        // no-jump trajectory's results (one entry, with
                              // psi), or all null: no shortcut
    int32_t*   zdone;         // set to 1 (release) once `zeroth` is complete
    int32_t    potential;     // QT_POTENTIAL_*
    int32_t    pad2;
    double     md_factor;     // KSU: Debye-mass factor
    const void* ksu_phi;      // KSU: (phi, phi') table, precision of the kernel
};

// Internal flag (above the public QT_FLAG_* bits): the group is the zeroth
// trajectory of a batch, threshold 0 (it never jumps; its smallest gap is its
// smallest norm).
constexpr int32_t kFlagZeroth = 1 << 16;

// Entry of exp(-2 pi i r k / L) in a level table of FFT twiddles (built by
// the host, read by PassTwiddles::load_level): levels L = 4, 8, ... in turn,
// each 7 L/2 entries: three rows of L/2 pairs (r, r + 1) = (1, 2), (3, 4),
// (5, 6), the pair of k at 2k, then the row r = 7 of L/2 entries k.  A table
// for FFTs of length up to n holds level_table_len(n) entries.
constexpr int level_index(int L, int r, int k)
{
    return 7 * (L - 4) / 2 + (r <= 6 ? ((r - 1) >> 1) * L + 2 * k + ((r - 1) & 1) : 3 * L + k);
}
constexpr int level_table_len(int n) { return level_index(2 * n, 1, 0); }
// Entry of the value at point m (m < n) of a table of length n held in
// mirror pairs (entry e < n/2: the values at e and n - e, at 0 and n/2 for
// e = 0; read by load_mirror_pairs), in complex elements.
constexpr int mirror_pair_index(int n, int m)
{
    return m < n / 2 ? 2 * m : (m == n / 2 ? 1 : 2 * (n - m) + 1);
}

struct FusedArgs {
    const GroupDesc* groups;
    const int32_t*   item_group;
    const int64_t*   item_index;
    int32_t          n_items;
    int32_t*         queue;
    const void*      tw;      // N complex: exp(-2 pi i m / N)
    const void*      prew;   // N complex: ((s+1/2)/2, (s-1/2)/2), s = sin(pi m / N)
    int64_t          seg_steps;   // <= 0: run to the end
};

// Kernel launchers (qt_kernels.hip).  Return hipSuccess or the launch error.
struct FusedKey { int prec; int N; int W; };
typedef hipError_t (*fused_launcher)(const FusedArgs&, int grid, hipStream_t s);
// Threads-per-trajectory candidates compiled for (precision, N); count returned.
int fused_variants(int prec, int N, int* W_out, int max_out);
fused_launcher fused_get(int prec, int N, int W);
// Occupancy of a variant: resident workgroups per CU.
int fused_occupancy(int prec, int N, int W);
// The variant compiled for the isotropic KSU potential at (precision, N):
// its block size, launcher and resident workgroups per CU.
bool fused_ksu_variant(int prec, int N, int* W, fused_launcher* launch, int* slots_per_cu);

hipError_t launch_queue_reset(int32_t* q, hipStream_t s);
// zeroes n int32 values (a fill kernel, safe under graph capture)
hipError_t launch_zero_i32(int32_t* p, int64_t n, hipStream_t s);
// complex values of the precision -> interleaved FP64 pairs
hipError_t launch_widen(const void* src, int prec, double* dst, int64_t count, hipStream_t s);

// Plain (unfused, FP64) form: one kernel per sub-step.
struct PlainArgs {
    const GroupDesc* g;       // one group
    double*    psi;           // n_traj * 2N doubles, natural order
    TrajState* st;
    int64_t    n_traj;
    int32_t    N;
    const void* tw;
    const void* prew;
};
hipError_t plain_init(const PlainArgs& a, hipStream_t s);
hipError_t plain_space(const PlainArgs& a, int64_t n, hipStream_t s);
hipError_t plain_dst(const PlainArgs& a, hipStream_t s);
hipError_t plain_kinetic(const PlainArgs& a, hipStream_t s);
hipError_t plain_norm_jump(const PlainArgs& a, int64_t n, hipStream_t s);
hipError_t plain_finalize(const PlainArgs& a, hipStream_t s);
bool plain_supported(int N);
// y = S (f .* (S x)) + d .* x for n_vec real vectors of length N (rows of x
// and y, device memory; d may be null), S the FP64 DST-I (qt_eigen.hip)
hipError_t eig_apply(int N, const double* x, double* y, int n_vec, const double* f,
                     const double* d, const void* tw, const void* prew, hipStream_t s);

}  // namespace qt
