// Exercises the host-only functions of librte (paper_2102_09038_amd/csrc/host.cpp) for the
// sanitizer build of tests/test_host_sanitize.py.  Reads the meshes the test writes (flat
// little-endian arrays from the seeded instance generator) and checks:
// - validate_problem accepts the instance and rejects broken copies with the right status;
// - pair_sphere finds half of the triangles, each with its antipode;
// - p1_pattern gives sorted rows, a symmetric pattern and the diagonal;
// - rcm is a permutation whose bandwidth does not exceed the natural order's;
// - sliced_ell holds every pattern entry exactly once;
// - band_cholesky reproduces random SPD band matrices (L L^T = A to 1e-12) and rejects an
//   indefinite one;
// - estimate_footprint orders its variants as the allocations do, at the realistic size.
// Prints "host_check ok" on success; any failed check exits with status 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "host.h"

namespace {

int g_fail = 0;
void check(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        g_fail = 1;
    }
}

template <typename T>
std::vector<T> read_array(const std::string& path) {
    std::ifstream f(path, std::ios::binary);
    f.seekg(0, std::ios::end);
    const size_t bytes = (size_t)f.tellg();
    f.seekg(0);
    std::vector<T> v(bytes / sizeof(T));
    f.read(reinterpret_cast<char*>(v.data()), (std::streamsize)bytes);
    return v;
}

struct Mesh {
    int dim = 2;
    std::vector<double> vert, sigma_t, sigma_s, svert, q;
    std::vector<int32_t> cell, stri;
    rte_problem_desc desc() const {
        rte_problem_desc D{};
        D.dim = dim;
        D.n_vert = (int)(vert.size() / dim);
        D.vert = vert.data();
        D.n_cell = (int)sigma_t.size();
        D.cell = cell.data();
        D.sigma_t = sigma_t.data();
        D.sigma_s = sigma_s.data();
        D.g = 0.8;
        D.n_svert = (int)(svert.size() / 3);
        D.svert = svert.data();
        D.n_stri = (int)(stri.size() / 3);
        D.stri = stri.data();
        D.q_nodal = q.data();
        D.g_inflow = nullptr;
        return D;
    }
};

Mesh load(const std::string& dir, const std::string& name, int dim) {
    Mesh m;
    m.dim = dim;
    m.vert = read_array<double>(dir + "/" + name + ".vert");
    m.cell = read_array<int32_t>(dir + "/" + name + ".cell");
    m.sigma_t = read_array<double>(dir + "/" + name + ".sigma_t");
    m.sigma_s = read_array<double>(dir + "/" + name + ".sigma_s");
    m.svert = read_array<double>(dir + "/" + name + ".svert");
    m.stri = read_array<int32_t>(dir + "/" + name + ".stri");
    m.q = read_array<double>(dir + "/" + name + ".q");
    return m;
}

rte_assemble_opts opts() {
    rte_assemble_opts o{};
    o.quad_level = 2;
    o.n_even = 0;
    o.n_odd = 5;
    o.e0_solver = RTE_E0_BANDED;
    o.mixed = 1;
    o.odd_eig = 1;
    o.coarse_solver = RTE_COARSE_AUTO;
    return o;
}

rte_status status_of(const rte_problem_desc& D, const rte_assemble_opts& o) {
    try {
        rte::validate_problem(&D, &o);
        rte::pair_sphere(&D);
        return RTE_OK;
    } catch (const rte::Error& e) {
        return e.status;
    }
}

// The multigrid hierarchy's host part: the meshes are lattices (and a vertex swap is not); the
// coarse pattern is the coarse lattice's P1 pattern (symmetric, sorted, diagonal present); the
// coarse class values equal the pattern entries of P^T C P formed densely by brute force, with
// P built independently from lattice coordinates (weight 1 at even vertices, 1/2 at the two ends
// of the coarse edge a fine vertex bisects).
void check_multigrid(const Mesh& mesh, const rte_problem_desc& D, const std::vector<int>& rp,
                     const std::vector<int>& ci) {
    const int d = D.dim, n = D.n_vert;
    const int m = rte::lattice_m(&D);
    check(m > 0 && (d == 2 ? m * m : m * m * m) == n, "lattice recognised");
    {
        std::vector<double> v(mesh.vert);
        std::swap(v[d * 1], v[d * 2]);
        std::swap(v[d * 1 + 1], v[d * 2 + 1]);
        rte_problem_desc B = D;
        B.vert = v.data();
        check(rte::lattice_m(&B) == 0, "swapped vertices are not a lattice");
        std::vector<int32_t> cell(mesh.cell);
        std::swap(cell[1], cell[2]);
        std::swap(cell[d + 1 + 0], cell[d + 1 + 3 % (d + 1)]);
        B = D;
        B.cell = cell.data();
        (void)rte::lattice_m(&B);      // any answer; only memory safety is checked here
    }
    const std::vector<int> sizes = rte::mg_level_sizes(m);
    check(sizes.size() >= 2, "at least two levels");
    // coarsen one level with two random classes on the fine pattern (only the in-pattern
    // entries are compared: for such matrices the rest of P^T C P need not vanish)
    const int ncls = 2, nnz = rp[n];
    std::vector<double> cls((size_t)ncls * nnz);
    unsigned long long st = 12345;
    for (double& x : cls) {
        st = st * 6364136223846793005ULL + 1442695040888963407ULL;
        x = (double)(st >> 11) / 9007199254740992.0 - 0.5;
    }
    const rte::MgHostLevel L = rte::mg_coarsen(d, m, ncls, rp, ci, cls);
    const int mc = L.m, nc = L.n;
    check(mc == sizes[1] && nc == (d == 2 ? mc * mc : mc * mc * mc), "coarse size");
    check((int)L.rp.size() == nc + 1 && L.rp[nc] == (int)L.ci.size() && (int)L.cls.size() == ncls * L.rp[nc],
          "coarse CSR shape");
    std::set<std::pair<int, int>> ent;
    for (int I = 0; I < nc; ++I) {
        bool diag = false;
        for (int e = L.rp[I]; e < L.rp[I + 1]; ++e) {
            if (e > L.rp[I]) check(L.ci[e] > L.ci[e - 1], "coarse rows sorted");
            diag |= L.ci[e] == I;
            ent.insert({I, L.ci[e]});
        }
        check(diag, "coarse diagonal present");
        check(L.rp[I + 1] - L.rp[I] <= (d == 2 ? 7 : 15), "coarse stencil width");
    }
    for (const auto& pr : ent) check(ent.count({pr.second, pr.first}) == 1, "coarse pattern symmetric");
    if (nc > 800) return;                 // the dense product below is for small lattices
    std::vector<double> P((size_t)n * nc, 0.0);
    for (int f = 0; f < n; ++f) {
        int c[3], lo = 0, hi = 0, mul = 1;
        for (int a = 0, v = f; a < d; ++a, v /= m) c[a] = v % m;
        for (int a = 0; a < d; ++a, mul *= mc) {
            lo += (c[a] / 2) * mul;
            hi += ((c[a] + 1) / 2) * mul;
        }
        if (lo == hi) P[(size_t)f * nc + lo] = 1.0;
        else P[(size_t)f * nc + lo] = P[(size_t)f * nc + hi] = 0.5;
    }
    double worst = 0.0, scale = 0.0;
    for (int c = 0; c < ncls; ++c) {
        std::vector<double> CP((size_t)n * nc, 0.0);       // C P
        for (int i = 0; i < n; ++i)
            for (int e = rp[i]; e < rp[i + 1]; ++e)
                for (int J = 0; J < nc; ++J) CP[(size_t)i * nc + J] += cls[(size_t)c * nnz + e] * P[(size_t)ci[e] * nc + J];
        for (int I = 0; I < nc; ++I)
            for (int e = L.rp[I]; e < L.rp[I + 1]; ++e) {
                const int J = L.ci[e];
                double v = 0.0;
                for (int f = 0; f < n; ++f) v += P[(size_t)f * nc + I] * CP[(size_t)f * nc + J];
                worst = std::max(worst, std::fabs(v - L.cls[(size_t)c * L.rp[nc] + e]));
                scale = std::max(scale, std::fabs(v));
            }
    }
    check(worst <= 1e-12 * std::max(scale, 1.0), "coarse class values are the pattern entries of P^T C P");
    std::printf("multigrid: lattice %d, levels %zu, coarse n %d nnz %d, worst |P^T C P - coarse| %.1e\n", m,
                sizes.size(), nc, L.rp[nc], worst);
}

void check_mesh(const Mesh& m, const char* name) {
    const rte_problem_desc D = m.desc();
    const rte_assemble_opts o = opts();
    check(status_of(D, o) == RTE_OK, name);
    // broken copies
    {
        rte_problem_desc B = D;
        B.g = 1.0;
        check(status_of(B, o) == RTE_E_PHYS, "g = 1 rejected");
        std::vector<double> ss(m.sigma_t);
        B = D;
        B.sigma_s = ss.data();
        check(status_of(B, o) == RTE_E_PHYS, "sigma_s = sigma_t rejected");
        std::vector<int32_t> cell(m.cell);
        cell[0] = D.n_vert;
        B = D;
        B.cell = cell.data();
        check(status_of(B, o) == RTE_E_MESH, "cell index out of range rejected");
        std::vector<double> sv(m.svert);
        sv[0] *= 2.0;
        B = D;
        B.svert = sv.data();
        check(status_of(B, o) == RTE_E_MESH, "non-unit sphere vertex rejected");
        B = D;
        B.n_stri -= 1;
        check(status_of(B, o) == RTE_E_MESH, "odd triangle count rejected");
        std::vector<double> q(m.q);
        q[1] = std::nan("");
        B = D;
        B.q_nodal = q.data();
        check(status_of(B, o) == RTE_E_ARG, "non-finite source rejected");
        rte_assemble_opts bo = o;
        bo.n_odd = 0;
        check(status_of(D, bo) == RTE_E_ARG, "n_odd = 0 rejected");
        check(status_of(D, bo) != RTE_OK, "bad options rejected");
    }
    // sphere pairing
    const std::vector<int> up = rte::pair_sphere(&D);
    check((int)up.size() * 2 == D.n_stri, "half of the triangles are upper");
    // pattern
    std::vector<int> rp, ci;
    rte::p1_pattern(&D, rp, ci);
    const int n = D.n_vert;
    check((int)rp.size() == n + 1 && rp[0] == 0 && rp[n] == (int)ci.size(), "CSR shape");
    std::set<std::pair<int, int>> ent;
    for (int i = 0; i < n; ++i) {
        bool diag = false;
        for (int e = rp[i]; e < rp[i + 1]; ++e) {
            if (e > rp[i]) check(ci[e] > ci[e - 1], "sorted rows");
            diag |= ci[e] == i;
            ent.insert({i, ci[e]});
        }
        check(diag, "diagonal present");
    }
    for (const auto& pr : ent) check(ent.count({pr.second, pr.first}) == 1, "symmetric pattern");
    // orders
    std::vector<int> ident(n);
    for (int i = 0; i < n; ++i) ident[i] = i;
    const std::vector<int> perm = rte::rcm(n, rp, ci);
    std::vector<int> seen(n, 0);
    for (int i = 0; i < n; ++i) {
        check(perm[i] >= 0 && perm[i] < n, "permutation range");
        if (perm[i] >= 0 && perm[i] < n) seen[perm[i]]++;
    }
    for (int i = 0; i < n; ++i) check(seen[i] == 1, "permutation is a bijection");
    check(rte::band_width(perm, rp, ci) <= rte::band_width(ident, rp, ci), "RCM does not widen the band");
    // the order of the band factors: the natural one unless RCM is more than 3% narrower, and
    // the returned width is that order's
    {
        std::vector<int> order;
        bool natural = false;
        const int bw = rte::band_order(n, rp, ci, order, &natural);
        const int bw_nat = rte::band_width(ident, rp, ci), bw_rcm = rte::band_width(perm, rp, ci);
        check(bw == rte::band_width(order, rp, ci), "band_order returns its order's width");
        check(natural == (100L * (bw_nat + 1) <= 103L * (bw_rcm + 1)), "natural order chosen within 3%");
        check(natural ? order == ident : order == perm, "band_order returns the chosen order");
    }
    // sliced ELL
    std::vector<int> sptr, col, epos;
    const size_t len = rte::sliced_ell(n, rp, ci, &sptr, &col, &epos);
    check(len == col.size() && len == epos.size() && len % 64 == 0, "ELL sizes");
    std::vector<int> hits(ci.size(), 0);
    for (size_t qd = 0; qd < len; ++qd) {
        check(col[qd] >= 0 && col[qd] < n, "ELL column range");
        if (epos[qd] >= 0) {
            hits[epos[qd]]++;
            check(col[qd] == ci[epos[qd]], "ELL column matches CSR");
        }
    }
    for (int h : hits) check(h == 1, "every CSR entry once in ELL");
    // footprint
    size_t peak = 0;
    const size_t b1 = rte::estimate_footprint(&D, &o, &peak);
    check(b1 > 0 && peak >= b1, "footprint positive");
    rte_assemble_opts o2 = o;
    o2.mixed = 2;
    size_t peak2 = 0;
    const size_t b2 = rte::estimate_footprint(&D, &o2, &peak2);
    check(b2 < b1 && peak2 > b2, "mixed = 2 drops the FP64 factors after assembly");
    rte_assemble_opts oc = o;
    oc.e0_solver = RTE_E0_CG;
    oc.mixed = 0;
    check(rte::estimate_footprint(&D, &oc, nullptr) > 0, "CG footprint");
    std::printf("%s: n_vert %d, nnz %zu, band %d -> %d, ELL %zu, footprint %zu bytes\n", name, n, ci.size(),
                rte::band_width(ident, rp, ci), rte::band_width(perm, rp, ci), len, b1);
    check_multigrid(m, D, rp, ci);
}

void check_band_cholesky() {
    std::mt19937_64 rng(7);
    std::uniform_real_distribution<double> u(-1.0, 1.0);
    for (int bw : {0, 1, 7, 40}) {
        const int n = 300;
        const size_t w1 = (size_t)bw + 1;
        std::vector<double> A(n * w1, 0.0);
        for (int i = 0; i < n; ++i) {
            for (int t = 0; t < bw; ++t)
                if (i - bw + t >= 0) A[i * w1 + t] = u(rng);
            A[i * w1 + bw] = 2.0 * bw + 1.0 + std::fabs(u(rng));   // diagonally dominant
        }
        std::vector<double> L(A);
        rte::band_cholesky(L, n, bw);
        double err = 0.0, nrm = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = std::max(0, i - bw); j <= i; ++j) {
                // (L L^T)(i, j) = sum_k L(i, k) L(j, k), diagonals stored as 1 / L(k, k)
                double s = 0.0;
                for (int kk = std::max(0, i - bw); kk <= j; ++kk) {
                    const double lik = kk == i ? 1.0 / L[i * w1 + bw] : L[i * w1 + bw + kk - i];
                    const double ljk = kk == j ? 1.0 / L[j * w1 + bw] : L[j * w1 + bw + kk - j];
                    s += lik * ljk;
                }
                const double a = A[i * w1 + bw + j - i];
                err = std::max(err, std::fabs(s - a));
                nrm = std::max(nrm, std::fabs(a));
            }
        check(err <= 1e-12 * nrm, "band Cholesky reproduces A");
    }
    std::vector<double> bad = {1.0, 0.0, 2.0, -5.0};   // [[1, 2], [2, -5]] lower band, bw = 1
    bool threw = false;
    try {
        rte::band_cholesky(bad, 2, 1);
    } catch (const rte::Error& e) {
        threw = e.status == RTE_E_ARG;
    }
    check(threw, "indefinite band matrix rejected");
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) {
        std::printf("usage: host_check <dir>\n");
        return 2;
    }
    const std::string dir = argv[1];
    check_mesh(load(dir, "grid2d", 2), "2D 128x128 squares, 2048 sphere triangles");
    check_mesh(load(dir, "grid3d", 3), "3D 8^3 cubes, 512 sphere triangles");
    check_band_cholesky();
    if (g_fail) return 1;
    std::printf("host_check ok\n");
    return 0;
}
