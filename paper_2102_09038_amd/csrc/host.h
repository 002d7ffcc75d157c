// Host-only parts of librte that need no GPU: errors, validation of a problem description,
// the antipodal pairing of the sphere mesh, the P1 pattern and its bandwidth-reducing order,
// the host band Cholesky, the sliced-ELL layout of the pattern, the arithmetic of the blocked
// band layout, and the prediction of a handle's device footprint.  Plain C++ with no HIP
// header, so that these functions can also be built with the address and undefined-behaviour
// sanitizers and exercised on a CPU (tests/sanitize/host_check.cpp).  The layout functions are
// constexpr, which also makes them callable from device code.
#pragma once

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rte.h"

namespace rte {

// ----------------------------------------------------------------------------- errors
struct Error : std::runtime_error {
    rte_status status;
    Error(rte_status s, const std::string& msg) : std::runtime_error(msg), status(s) {}
};

[[noreturn]] inline void fail(rte_status s, const std::string& msg) { throw Error(s, msg); }

constexpr int kMaxClasses = 16;                         // sparse value classes of the P1 pattern
constexpr double kEcinvMaxBytes = 12.0 * (1 << 30);     // budget of an explicit E_c^{-1}
constexpr int kFacCols = 9;     // columns per thread of the band factorisation's trailing update
// Chebyshev steps whose coefficients are tabulated per multigrid level and direction (at least
// the steps of a smoothing pass on any level)
constexpr int kMgChebSteps = 8;

namespace k {
// Blocked band layout of a factor with band width bw (kernels_band.hip): rows in blocks of
// 64, band offsets t = 0..bw in groups of vec consecutive entries (vec = 16 bytes / element);
// a row block holds G = H P groups (the solve kernel's ring depth H times its phase count P,
// with H P >= ceil((bw+1)/vec)), zero past t = bw.  The shapes the solve kernel is built for
// have distinct H P, so a layout's group count G names its shape.  band_shape picks the
// default (little padding, then a deeper ring); the autotuner may choose another.
struct BandShape {
    int H, P;
};
constexpr int kBandShapes = 9;
constexpr BandShape band_shape_at(int k) {
    const int hs[kBandShapes] = {9, 17, 33, 9, 17, 33, 17, 33, 33};
    const int ps[kBandShapes] = {1, 1, 1, 2, 2, 2, 3, 3, 4};
    return BandShape{hs[k], ps[k]};
}
constexpr BandShape band_shape(int bw, int vec) {
    const int g = (bw + vec) / vec;
    BandShape best{0, 0};
    int waste = 1 << 30;
    for (int k = 0; k < kBandShapes; ++k) {
        const BandShape sh = band_shape_at(k);
        const int cap = sh.H * sh.P;
        if (cap < g) continue;
        // prefer little padding, then a deeper ring
        const int w = (cap - g) * 4 - sh.H;
        if (w < waste) {
            waste = w;
            best = sh;
        }
    }
    return best;
}
// the shape of a layout with G groups per row block ({0, 0}: none)
constexpr BandShape band_shape_of_groups(int G) {
    for (int k = 0; k < kBandShapes; ++k) {
        const BandShape sh = band_shape_at(k);
        if (sh.H * sh.P == G) return sh;
    }
    return BandShape{0, 0};
}
// default group count (0 if the band is too wide for every shape)
constexpr size_t band_groups(int bw, int vec) {
    const BandShape sh = band_shape(bw, vec);
    return (size_t)sh.H * sh.P;
}
constexpr size_t band_blk_index_g(int r, int t, int G, int vec) {
    return (((size_t)(r >> 6) * G + t / vec) * 64 + (r & 63)) * vec + t % vec;
}
constexpr size_t band_blk_size_g(int n, int G, int vec) { return (size_t)((n + 63) / 64) * G * 64 * vec; }
// the same in the default layout
constexpr size_t band_blk_index(int r, int t, int bw, int vec) {
    return band_blk_index_g(r, t, (int)band_groups(bw, vec), vec);
}
// number of elements of one system's factor in the default layout (0 if the band is too wide)
constexpr size_t band_blk_size(int n, int bw, int vec) { return band_blk_size_g(n, (int)band_groups(bw, vec), vec); }
// whether the device band factorisation (an LDS window of (bw+1)^2 FP64 values, at most
// 150 KiB) takes half-bandwidth bw
constexpr bool band_factor_fits(int bw) {
    return (size_t)(bw + 1) * (bw + 1) * sizeof(double) <= 150 * 1024 && bw + 1 <= 16 * kFacCols;
}
}  // namespace k

// Checks every field of a problem description and its assembly options (Sec. 1 data, Sec. 2
// parameter assumptions 0 <= g < 1, sigma_t > 0, max sigma_s / sigma_t < 1; Sec. 4 meshes)
// before any device work; throws Error.  Returns c = max sigma_s / sigma_t.
double validate_problem(const rte_problem_desc* D, const rte_assemble_opts* o);

// The triangles of the sphere mesh whose centroid lies in the upper half-sphere (z > 0, ties
// broken on y, then x), in mesh order; throws Error (RTE_E_MESH) unless every one has its
// antipode in the mesh and they are exactly half of the triangles (Sec. 4 even basis).
std::vector<int> pair_sphere(const rte_problem_desc* D);

// The P1 pattern of the spatial mesh: CSR rows rp (n_vert + 1) with sorted columns ci,
// diagonal included.
void p1_pattern(const rte_problem_desc* D, std::vector<int>& rp, std::vector<int>& ci);

// Half-bandwidth of the pattern in the order perm (perm[i] = new position of vertex i).
int band_width(const std::vector<int>& perm, const std::vector<int>& rp, const std::vector<int>& ci);

// Reverse Cuthill-McKee order of the pattern graph; returns perm[i] = new position of vertex i.
std::vector<int> rcm(int n, const std::vector<int>& rp, const std::vector<int>& ci);
// The vertex order of the band factors: the given (natural) order unless reverse Cuthill-McKee
// narrows the band by more than 3% (the natural order spares E_0^{-1} its two permutation
// passes over the vectors, which cost more than a 3% wider band).  Returns the band width;
// perm[i] = position of vertex i; *identity tells whether perm is the natural order.
int band_order(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>& perm,
               bool* identity);

// In place Cholesky factorisation L L^T = A of an SPD band matrix stored as its lower band by
// rows, A[i (bw+1) + bw + j - i] for j in [i - bw, i]; afterwards the diagonal entries hold
// 1 / L(i,i).  Throws Error (RTE_E_ARG) on a non-positive pivot.
void band_cholesky(std::vector<double>& A, int n, int bw);

// The pattern in sliced ELL form (slices of 64 rows, as many slots as the slice's longest row,
// slot j of a slice one contiguous group of 64 entries, lane = row): sptr[s] = first slot
// group of slice s, col = column of every entry (the row itself on padding), epos = the entry's
// CSR position (-1 on padding).  Returns the number of entries; arrays filled when non-null.
size_t sliced_ell(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>* sptr,
                  std::vector<int>* col, std::vector<int>* epos);

// ---- geometric multigrid for the E_0 blocks on lattice meshes (multigrid remark of Sec. 5.5)
// The mesh is the Freudenthal (Kuhn) triangulation of a box when its vertices are the points of
// an m^d lattice numbered i + m (j + m k) and every cell edge joins lattice points whose
// difference has entries in {0, 1}.  Returns m, or 0 for any other mesh.
int lattice_m(const rte_problem_desc* D);
// Vertices per axis of the levels, finest first: a level is added while the cell count per
// axis is even and at least 4.
std::vector<int> mg_level_sizes(int m);
// One coarse level: the P1 pattern of its lattice (CSR, sorted columns) and the Galerkin
// products P^T C_c P of the finer level's value classes C_c ([ncls * nnz]); P is the P1
// interpolant between the nested lattices.  The entries outside the coarse P1 pattern are
// exact zeros (the supports of two coarse basis functions that share no coarse cell meet in
// a null set) and are not formed.
struct MgHostLevel {
    int m = 0, n = 0;
    std::vector<int> rp, ci;
    std::vector<double> cls;
};
MgHostLevel mg_coarsen(int d, int m, int ncls, const std::vector<int>& rp, const std::vector<int>& ci,
                       const std::vector<double>& cls);

// Device bytes a handle of this problem holds once assembled with o and given the workspace
// of a solve, and the peak during assembly (*peak, nullable).  Host work only.
size_t estimate_footprint(const rte_problem_desc* D, const rte_assemble_opts* o, size_t* peak);

}  // namespace rte
