// Host-only parts of librte (declared in host.h): no HIP, so that a sanitizer build can run
// them on a CPU.  See host.h for what each function computes.
#include "host.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <deque>
#include <map>
#include <numeric>

namespace rte {

double validate_problem(const rte_problem_desc* D, const rte_assemble_opts* o) {
    if (!D || !o) fail(RTE_E_ARG, "null descriptor or options");
    if (o->mixed < 0 || o->mixed > 2) fail(RTE_E_ARG, "mixed must be 0, 1 or 2");
    if (o->odd_eig != 0 && o->odd_eig != 1) fail(RTE_E_ARG, "odd_eig must be 0 or 1");
    if (o->coarse_solver < RTE_COARSE_AUTO || o->coarse_solver > RTE_COARSE_QUICK)
        fail(RTE_E_ARG, "unknown coarse solver");
    const int d = D->dim;
    if (d != 2 && d != 3) fail(RTE_E_ARG, "dim must be 2 or 3");
    if (D->n_vert < d + 1 || D->n_cell < 1 || !D->vert || !D->cell) fail(RTE_E_ARG, "empty spatial mesh");
    if (!D->sigma_t || !D->sigma_s || !D->q_nodal) fail(RTE_E_ARG, "null sigma_t / sigma_s / q_nodal");
    if (D->g_inflow) fail(RTE_E_ARG, "inflow boundary data is not supported (vacuum boundary only)");
    if (D->n_stri < 2 || D->n_stri % 2 || !D->svert || !D->stri || D->n_svert < 3)
        fail(RTE_E_MESH, "sphere mesh must have an even, positive number of triangles");
    if (!(D->g >= 0.0 && D->g < 1.0)) fail(RTE_E_PHYS, "g must lie in [0, 1)");
    if (o->quad_level < 0 || o->quad_level > 6) fail(RTE_E_ARG, "quad_level must lie in 0..6");
    if (o->n_even < 0 || o->n_even > 8) fail(RTE_E_ARG, "n_even must lie in 0..8");
    if (o->n_odd < 1 || o->n_odd > 8) fail(RTE_E_ARG, "n_odd must lie in 1..8");
    const int nRp = D->n_vert, nRm = D->n_cell;
    double cmax = 0.0;
    for (int j = 0; j < nRm; ++j) {
        const double st = D->sigma_t[j], ss = D->sigma_s[j];
        if (!std::isfinite(st) || !std::isfinite(ss) || !(st > 0) || ss < 0)
            fail(RTE_E_PHYS, "sigma_t must be > 0 and sigma_s >= 0 (finite) in every cell");
        cmax = std::max(cmax, ss / st);
    }
    if (!(cmax < 1.0)) fail(RTE_E_PHYS, "max sigma_s/sigma_t must be < 1 (absorbing medium)");
    for (int i = 0; i < nRp * d; ++i)
        if (!std::isfinite(D->vert[i])) fail(RTE_E_ARG, "non-finite vertex coordinate");
    for (int i = 0; i < nRp; ++i)
        if (!std::isfinite(D->q_nodal[i])) fail(RTE_E_ARG, "non-finite source value");
    for (int i = 0; i < nRm * (d + 1); ++i)
        if (D->cell[i] < 0 || D->cell[i] >= nRp) fail(RTE_E_MESH, "cell vertex index out of range");
    for (int i = 0; i < D->n_stri * 3; ++i)
        if (D->stri[i] < 0 || D->stri[i] >= D->n_svert) fail(RTE_E_MESH, "sphere vertex index out of range");
    for (int i = 0; i < D->n_svert; ++i) {
        const double* v = D->svert + 3 * i;
        const double nv = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(std::fabs(nv - 1.0) < 1e-10)) fail(RTE_E_MESH, "sphere vertices must be unit vectors");
    }
    return cmax;
}

std::vector<int> pair_sphere(const rte_problem_desc* D) {
    const int nt = D->n_stri;
    auto vkey = [](const double* v) {
        auto q = [](double x) { return (long long)std::llround(x * 1e9); };
        return std::array<long long, 3>{q(v[0]), q(v[1]), q(v[2])};
    };
    std::map<std::array<long long, 9>, int> trikey;
    auto tkey = [&](const int* t, double sign) {
        std::array<std::array<long long, 3>, 3> ks;
        for (int v = 0; v < 3; ++v) {
            const double* p = D->svert + 3 * t[v];
            const double q[3] = {sign * p[0], sign * p[1], sign * p[2]};
            ks[v] = vkey(q);
        }
        std::sort(ks.begin(), ks.end());
        std::array<long long, 9> out;
        for (int v = 0; v < 3; ++v)
            for (int e = 0; e < 3; ++e) out[3 * v + e] = ks[v][e];
        return out;
    };
    for (int t = 0; t < nt; ++t) trikey[tkey(D->stri + 3 * t, 1.0)] = t;
    std::vector<int> upper;
    for (int t = 0; t < nt; ++t) {
        double cz = 0, cy = 0, cx = 0;
        for (int v = 0; v < 3; ++v) {
            const double* p = D->svert + 3 * D->stri[3 * t + v];
            cx += p[0]; cy += p[1]; cz += p[2];
        }
        const double key = cz != 0 ? cz : (cy != 0 ? cy : cx);
        if (key > 0) {
            if (!trikey.count(tkey(D->stri + 3 * t, -1.0)))
                fail(RTE_E_MESH, "sphere triangle " + std::to_string(t) + " has no antipodal partner");
            upper.push_back(t);
        }
    }
    if ((int)upper.size() * 2 != nt) fail(RTE_E_MESH, "sphere mesh is not split evenly into antipodal pairs");
    return upper;
}

void p1_pattern(const rte_problem_desc* D, std::vector<int>& rp, std::vector<int>& ci) {
    const int d = D->dim, nv = d + 1, nRp = D->n_vert, nRm = D->n_cell;
    std::vector<std::vector<int>> adj(nRp);
    for (int j = 0; j < nRm; ++j)
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) adj[D->cell[nv * j + a]].push_back(D->cell[nv * j + b]);
    rp.assign(nRp + 1, 0);
    ci.clear();
    for (int i = 0; i < nRp; ++i) {
        auto& v = adj[i];
        v.push_back(i);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        rp[i + 1] = rp[i] + (int)v.size();
        ci.insert(ci.end(), v.begin(), v.end());
    }
}

int band_width(const std::vector<int>& perm, const std::vector<int>& rp, const std::vector<int>& ci) {
    int bw = 0;
    for (size_t i = 0; i + 1 < rp.size(); ++i)
        for (int e = rp[i]; e < rp[i + 1]; ++e) bw = std::max(bw, std::abs(perm[i] - perm[ci[e]]));
    return bw;
}

// reverse Cuthill-McKee on the P1 graph; returns perm[i] = new position of vertex i
std::vector<int> rcm(int n, const std::vector<int>& rp, const std::vector<int>& ci) {
    std::vector<int> deg(n), order;
    order.reserve(n);
    for (int i = 0; i < n; ++i) deg[i] = rp[i + 1] - rp[i];
    std::vector<char> seen(n, 0);
    std::vector<int> byDeg(n);
    std::iota(byDeg.begin(), byDeg.end(), 0);
    std::stable_sort(byDeg.begin(), byDeg.end(), [&](int a, int b) { return deg[a] < deg[b]; });
    for (int start : byDeg) {
        if (seen[start]) continue;
        std::deque<int> dq{start};
        seen[start] = 1;
        while (!dq.empty()) {
            const int v = dq.front();
            dq.pop_front();
            order.push_back(v);
            std::vector<int> nb;
            for (int e = rp[v]; e < rp[v + 1]; ++e)
                if (!seen[ci[e]]) { seen[ci[e]] = 1; nb.push_back(ci[e]); }
            std::stable_sort(nb.begin(), nb.end(), [&](int a, int b) { return deg[a] < deg[b]; });
            for (int u : nb) dq.push_back(u);
        }
    }
    std::reverse(order.begin(), order.end());
    std::vector<int> perm(n);
    for (int p = 0; p < n; ++p) perm[order[p]] = p;
    return perm;
}

int band_order(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>& perm,
               bool* identity) {
    std::vector<int> ident(n);
    std::iota(ident.begin(), ident.end(), 0);
    const int bw_nat = band_width(ident, rp, ci);
    std::vector<int> r = rcm(n, rp, ci);
    const int bw_rcm = band_width(r, rp, ci);
    const bool nat = 100 * ((long)bw_nat + 1) <= 103 * ((long)bw_rcm + 1);
    perm = nat ? std::move(ident) : std::move(r);
    if (identity) *identity = nat;
    return nat ? bw_nat : bw_rcm;
}

void band_cholesky(std::vector<double>& A, int n, int bw) {
    const size_t w1 = (size_t)bw + 1;
    for (int j = 0; j < n; ++j) {
        double* rj = A.data() + w1 * j;
        double s = rj[bw];
        for (int k = std::max(0, j - bw); k < j; ++k) { const double v = rj[bw + k - j]; s -= v * v; }
        if (!(s > 0)) fail(RTE_E_ARG, "coarse matrix is not positive definite");
        const double ljj = std::sqrt(s);
        rj[bw] = ljj;
        const int i1 = std::min(n - 1, j + bw);
        for (int i = j + 1; i <= i1; ++i) {
            double* ri = A.data() + w1 * i;
            double t = ri[bw + j - i];
            const int k0 = std::max(0, i - bw);
            for (int k = k0; k < j; ++k) t -= ri[bw + k - i] * rj[bw + k - j];
            ri[bw + j - i] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i) A[w1 * i + bw] = 1.0 / A[w1 * i + bw];
}

size_t sliced_ell(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>* sptr,
                  std::vector<int>* col, std::vector<int>* epos) {
    const int nslice = (n + 63) / 64;
    std::vector<int> sp(nslice + 1, 0);
    for (int sl = 0; sl < nslice; ++sl) {
        int w = 0;
        for (int i = 64 * sl; i < std::min(n, 64 * sl + 64); ++i) w = std::max(w, rp[i + 1] - rp[i]);
        sp[sl + 1] = sp[sl] + w;
    }
    const size_t len = (size_t)sp[nslice] * 64;
    if (col && epos) {
        col->assign(len, 0);
        epos->assign(len, -1);
        for (int sl = 0; sl < nslice; ++sl)
            for (int j = 0; j < sp[sl + 1] - sp[sl]; ++j)
                for (int lane = 0; lane < 64; ++lane) {
                    const int i = 64 * sl + lane;
                    const size_t q = ((size_t)sp[sl] + j) * 64 + lane;
                    if (i < n && j < rp[i + 1] - rp[i]) {
                        (*epos)[q] = rp[i] + j;
                        (*col)[q] = ci[rp[i] + j];
                    } else {
                        (*col)[q] = i < n ? i : 0;
                    }
                }
    }
    if (sptr) *sptr = sp;
    return len;
}

int lattice_m(const rte_problem_desc* D) {
    const int d = D->dim, nv = D->n_vert;
    int m = (int)std::lround(std::pow((double)nv, 1.0 / d));
    while (m > 1 && (d == 2 ? m * m : m * m * m) > nv) --m;
    while ((d == 2 ? (m + 1) * (m + 1) : (m + 1) * (m + 1) * (m + 1)) <= nv) ++m;
    if (m < 2 || (d == 2 ? m * m : m * m * m) != nv) return 0;
    double lo[3], hi[3];
    for (int a = 0; a < d; ++a) {
        lo[a] = D->vert[a];
        hi[a] = D->vert[(size_t)(nv - 1) * d + a];
        if (!(hi[a] > lo[a])) return 0;
    }
    for (int v = 0; v < nv; ++v) {
        int c = v;
        for (int a = 0; a < d; ++a, c /= m) {
            const double x = lo[a] + (hi[a] - lo[a]) * (c % m) / (m - 1);
            if (std::fabs(D->vert[(size_t)v * d + a] - x) > 1e-12 * std::max(1.0, std::fabs(hi[a] - lo[a]))) return 0;
        }
    }
    // every cell edge: lattice offset with entries in {0, 1} from its smaller-indexed end
    const int nvc = d + 1;
    if (D->n_cell != (d == 2 ? 2 : 6) * (int)std::pow(m - 1, d)) return 0;
    for (int j = 0; j < D->n_cell; ++j)
        for (int a = 0; a < nvc; ++a)
            for (int b = 0; b < nvc; ++b) {
                int u = D->cell[nvc * j + a], w = D->cell[nvc * j + b];
                if (u >= w) continue;
                for (int t = 0; t < d; ++t, u /= m, w /= m) {
                    const int off = w % m - u % m;
                    if (off != 0 && off != 1) return 0;
                }
            }
    return m;
}

std::vector<int> mg_level_sizes(int m) {
    std::vector<int> out{m};
    while ((out.back() - 1) % 2 == 0 && out.back() - 1 >= 4) out.push_back((out.back() - 1) / 2 + 1);
    return out;
}

MgHostLevel mg_coarsen(int d, int m, int ncls, const std::vector<int>& rp, const std::vector<int>& ci,
                       const std::vector<double>& cls) {
    MgHostLevel L;
    L.m = (m - 1) / 2 + 1;
    const int mc = L.m;
    const int nc = d == 2 ? mc * mc : mc * mc * mc;
    L.n = nc;
    const int nnz_f = rp.back();
    auto coords = [&](int v, int mm, int* c) {
        for (int a = 0; a < d; ++a, v /= mm) c[a] = v % mm;
    };
    auto index = [&](const int* c, int mm) {
        int v = 0;
        for (int a = d - 1; a >= 0; --a) v = v * mm + c[a];
        return v;
    };
    // the coarse P1 pattern: I and I +- e_S for every nonempty axis set S, in bounds
    const int nsets = (1 << d) - 1;
    L.rp.assign(nc + 1, 0);
    std::vector<std::vector<int>> rows(nc);
    for (int I = 0; I < nc; ++I) {
        int c[3];
        coords(I, mc, c);
        std::vector<int>& r = rows[I];
        r.push_back(I);
        for (int S = 1; S <= nsets; ++S)
            for (int sg = -1; sg <= 1; sg += 2) {
                int q[3];
                bool in = true;
                for (int a = 0; a < d; ++a) {
                    q[a] = c[a] + ((S >> a) & 1) * sg;
                    in = in && q[a] >= 0 && q[a] < mc;
                }
                if (in) r.push_back(index(q, mc));
            }
        std::sort(r.begin(), r.end());
        L.rp[I + 1] = L.rp[I] + (int)r.size();
    }
    L.ci.resize(L.rp[nc]);
    for (int I = 0; I < nc; ++I) std::copy(rows[I].begin(), rows[I].end(), L.ci.begin() + L.rp[I]);
    const int nnz_c = L.rp[nc];
    L.cls.assign((size_t)ncls * nnz_c, 0.0);
    // coarse parents of fine vertex f with their weights (1 at an even vertex, else 1/2 at the
    // two ends of the coarse edge f bisects)
    auto parents = [&](int f, int* pv, double* pw) {
        int c[3], lo[3], hi[3];
        coords(f, m, c);
        for (int a = 0; a < d; ++a) {
            lo[a] = c[a] / 2;
            hi[a] = (c[a] + 1) / 2;
        }
        const int il = index(lo, mc), ih = index(hi, mc);
        if (il == ih) {
            pv[0] = il;
            pw[0] = 1.0;
            return 1;
        }
        pv[0] = il; pw[0] = 0.5;
        pv[1] = ih; pw[1] = 0.5;
        return 2;
    };
    for (int I = 0; I < nc; ++I) {
        int c[3];
        coords(I, mc, c);
        // the fine vertices coarse vertex I interpolates to, with weights: 2I, and 2I +- e_S
        int fv[32];
        double fw[32];
        int nf = 0;
        {
            int q[3];
            for (int a = 0; a < d; ++a) q[a] = 2 * c[a];
            fv[nf] = index(q, m);
            fw[nf++] = 1.0;
        }
        for (int S = 1; S <= nsets; ++S)
            for (int sg = -1; sg <= 1; sg += 2) {
                int q[3];
                bool in = true;
                for (int a = 0; a < d; ++a) {
                    q[a] = 2 * c[a] + ((S >> a) & 1) * sg;
                    in = in && q[a] >= 0 && q[a] < m;
                }
                if (in) {
                    fv[nf] = index(q, m);
                    fw[nf++] = 0.5;
                }
            }
        const int* cb = L.ci.data() + L.rp[I];
        const int* ce = L.ci.data() + L.rp[I + 1];
        for (int t = 0; t < nf; ++t) {
            const int f = fv[t];
            for (int e = rp[f]; e < rp[f + 1]; ++e) {
                int pv[2];
                double pw[2];
                const int np = parents(ci[e], pv, pw);
                for (int u = 0; u < np; ++u) {
                    const int* hit = std::lower_bound(cb, ce, pv[u]);
                    if (hit == ce || *hit != pv[u]) continue;    // an exact zero outside the pattern
                    const size_t ec = (size_t)(hit - L.ci.data());
                    const double w = fw[t] * pw[u];
                    for (int cc = 0; cc < ncls; ++cc)
                        L.cls[(size_t)cc * nnz_c + ec] += w * cls[(size_t)cc * nnz_f + e];
                }
            }
        }
    }
    return L;
}

size_t estimate_footprint(const rte_problem_desc* D, const rte_assemble_opts* o, size_t* peak) {
    if (!D || !o) fail(RTE_E_ARG, "null descriptor or options");
    const int d = D->dim;
    if (d != 2 && d != 3) fail(RTE_E_ARG, "dim must be 2 or 3");
    if (D->n_vert < d + 1 || D->n_cell < 1 || !D->cell || D->n_stri < 2) fail(RTE_E_ARG, "empty mesh");
    const int nv = d + 1, nRp = D->n_vert, nRm = D->n_cell;
    const size_t nS = (size_t)D->n_stri / 2, nSm = 3 * nS;
    const size_t dN = (size_t)(o->n_even + 1) * (o->n_even + 2) / 2;
    const size_t dNm = (size_t)(o->n_odd + 1) * (o->n_odd + 2) / 2;
    std::vector<std::vector<int>> adj(nRp);
    for (int j = 0; j < nRm; ++j)
        for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
                const int va = D->cell[nv * j + a], vb = D->cell[nv * j + b];
                if (va < 0 || va >= nRp || vb < 0 || vb >= nRp) fail(RTE_E_MESH, "cell vertex out of range");
                adj[va].push_back(vb);
            }
    std::vector<int> rp(nRp + 1, 0), ci;
    for (int i = 0; i < nRp; ++i) {
        auto& v = adj[i];
        v.push_back(i);
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        rp[i + 1] = rp[i] + (int)v.size();
        ci.insert(ci.end(), v.begin(), v.end());
    }
    std::vector<int> order;
    const int sbw = band_order(nRp, rp, ci, order, nullptr);
    const size_t nnz = (size_t)rp[nRp], nc = dN * nRp, even = (size_t)nRp * nS;
    const size_t cbw = dN * sbw + dN - 1;
    size_t b = 0;
    // angular operators: S+, S-, eigenbases (full odd basis twice), H, condensed G, moments;
    // without the odd eigendecomposition (uniform ratio, odd_eig = 0) neither odd basis
    bool uniform = true;
    if (D->sigma_t && D->sigma_s) {
        double lo = 1e300, hi = -1e300;
        for (int j = 0; j < nRm; ++j) {
            const double r = D->sigma_s[j] / D->sigma_t[j];
            lo = std::min(lo, r);
            hi = std::max(hi, r);
        }
        uniform = hi - lo <= 1e-13 * std::max(hi, 1e-300);
    }
    if (o->odd_eig == 0 && uniform) b += (nS * nS + 2 * nSm * nSm + nS * dN + 4 * nSm + 16 * nS) * 8;
    else b += (nS * nS + 4 * nSm * nSm + nSm * dNm + nS * dN + 4 * nSm + 16 * nS) * 8;
    b += (size_t)d * nS * d * nS * 8;
    // spatial data: cells, gradients, pattern values per class, incidence, source
    b += (size_t)nRm * (nv * 4 + nv * d * 8 + 4 * 8) + nnz * (4 + 8 * (kMaxClasses + 4)) + (size_t)nRp * 16;
    b += (size_t)nRm * nv * (4 + 4 + d * 8) + nS * kMaxClasses * 8 * 3 + even * 8;
    // coarse solve: explicit inverse or band factors
    size_t transient = 0;
    {
        const bool inv_fits = (double)nc * nc * 8 <= kEcinvMaxBytes, band_fits = k::band_groups((int)cbw, 2) != 0;
        int how = o->coarse_solver;
        if (how == RTE_COARSE_QUICK)
            how = (band_fits && k::band_factor_fits((int)cbw)) ? RTE_COARSE_BAND : RTE_COARSE_BLOCK;
        if (how == RTE_COARSE_AUTO) how = inv_fits ? RTE_COARSE_INVERSE : band_fits ? RTE_COARSE_BAND : RTE_COARSE_BLOCK;
        if (how == RTE_COARSE_INVERSE) {
            b += nc * nc * 8;
        } else if (how == RTE_COARSE_BAND) {
            b += 2 * k::band_blk_size((int)nc, (int)cbw, 2) * 8;
        } else {
            const size_t bs = std::max<size_t>(cbw, 1), nbk = (nc + bs - 1) / bs;
            b += (4 * nbk - 2) * bs * bs * 8 + 2 * nbk * bs * 8;
            transient = std::max(transient, nc * (cbw + 1) * 8);   // the band on its way to the blocks
        }
    }
    if (o->e0_solver == RTE_E0_BANDED) {
        const size_t f64 = 2 * k::band_blk_size(nRp, sbw, 2) * nS * 8;
        if (o->mixed != 2) b += f64;
        else transient = f64;
        if (o->mixed) b += 2 * k::band_blk_size(nRp, sbw, 4) * nS * 4;
    }
    if (o->mixed) b += (nS * nS + nSm * nSm) * 4 + (size_t)d * nS * d * nS * 2;
    b += nS * (size_t)(d * (d + 1) / 2) * 8;      // diagonal blocks of the condensed operator
    // the sliced ELL pattern; with the CG solver the explicit values (FP64, and FP32 when mixed),
    // inverse diagonals, three CG vectors and the per-tile partials
    const size_t ell = sliced_ell(nRp, rp, ci, nullptr, nullptr, nullptr);
    b += ell * 8 + ((size_t)nRp / 64 + 2) * 4;
    if (o->e0_solver == RTE_E0_CG || o->e0_solver == RTE_E0_MG) {
        const size_t ntiles = ((size_t)nRp + 255) / 256;
        b += 3 * even * 8 + 4 * nS * ntiles * 8 + 3 * nS * 8 + (nS + 1) * 4;
        if (o->mixed != 2) b += nS * ell * 8 + even * 8;
        if (o->mixed) b += nS * ell * 4 + even * 4;
    }
    if (o->e0_solver == RTE_E0_MG) {
        // per level: smoother values (FP32 for FP64 solves, BF16 for mixed ones), inverse
        // diagonals, Chebyshev intervals and coefficients per precision, five work vectors; levels 1..: the
        // sliced-ELL pattern (P1 stencil widths 7 / 15) and class values
        const int m = lattice_m(D);
        if (m) {
            const std::vector<int> sizes = mg_level_sizes(m);
            const size_t per = (o->mixed != 2 ? 8 : 0) + (o->mixed ? 4 : 0);
            const size_t sv = (o->mixed != 2 ? 4 : 0) + (o->mixed ? 2 : 0);
            const size_t w = d == 2 ? 7 : 15;
            for (size_t l = 0; l < sizes.size(); ++l) {
                const size_t nl = d == 2 ? (size_t)sizes[l] * sizes[l] : (size_t)sizes[l] * sizes[l] * sizes[l];
                const size_t len = (nl + 63) / 64 * 64 * w;
                b += nS * nl * per + 2 * nS * (1 + kMgChebSteps) * 8 * 2 + 5 * nl * nS * 8 + nS * len * sv;
                if (l > 0) b += 2 * len * 4 + (nl / 64 + 2) * 4 + (size_t)kMaxClasses * nl * w * 8;
            }
        }
    }
    // solver workspace: two odd-sized buffers, eleven even vectors, coarse vectors, reductions
    b += 2 * (size_t)nRm * nSm * 8 + 11 * even * 8 + 2 * nc * 8 + (1 << 16);
    if (peak) *peak = b + transient;
    return b;
}

}  // namespace rte
