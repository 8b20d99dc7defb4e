// Host-side mesh preprocessing and reference tables for the gfx950 DG library.
//
// Mesh input follows section 2.1 of Uzunca & Karasozen (arXiv:1502.02941):
// node coordinates, counter-clockwise element triples and the Dirichlet /
// Neumann boundary edge lists.  This file builds the edge connectivity
// (interior edges shared by exactly two elements, boundary edges classified by
// the two lists), the BSR block pattern (one dense block per coupled element
// pair), the per-element neighbour tables the assembly kernels read, and the
// reference quadrature / basis tables.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>

#include "dg_internal.h"

namespace dg {

// ---------------------------------------------------------------------------
// Quadrature: Golub-Welsch.  The nodes of the n-point Gauss-Jacobi rule are
// the eigenvalues of the symmetric tridiagonal Jacobi matrix of the monic
// recurrence; the weights are mu0 * (first eigenvector component)^2.  The
// eigenproblem is solved with cyclic Jacobi rotations (n <= 8 here).
// ---------------------------------------------------------------------------
static void sym_eig_jacobi(int n, double* A, double* V)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
        if (off < 1e-64) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < n; ++r) {  // columns p, q
                    double arp = A[r * n + p], arq = A[r * n + q];
                    A[r * n + p] = c * arp - s * arq;
                    A[r * n + q] = s * arp + c * arq;
                }
                for (int r = 0; r < n; ++r) {  // rows p, q
                    double apr = A[p * n + r], aqr = A[q * n + r];
                    A[p * n + r] = c * apr - s * aqr;
                    A[q * n + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < n; ++r) {
                    double vrp = V[r * n + p], vrq = V[r * n + q];
                    V[r * n + p] = c * vrp - s * vrq;
                    V[r * n + q] = s * vrp + c * vrq;
                }
            }
    }
}

void gauss_jacobi_gw(int n, double a, double b, double* x, double* w)
{
    std::vector<double> J(n * n, 0.0), V(n * n);
    for (int i = 0; i < n; ++i) {
        double s = 2.0 * i + a + b;
        J[i * n + i] = (i == 0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (s * (s + 2.0));
        if (i + 1 < n) {
            double k = i + 1.0, t = 2.0 * k + a + b;
            double off = std::sqrt(4.0 * k * (k + a) * (k + b) * (k + a + b) / (t * t * (t + 1.0) * (t - 1.0)));
            J[i * n + i + 1] = J[(i + 1) * n + i] = off;
        }
    }
    sym_eig_jacobi(n, J.data(), V.data());
    const double mu0 = std::pow(2.0, a + b + 1.0) * std::tgamma(a + 1.0) * std::tgamma(b + 1.0) / std::tgamma(a + b + 2.0);
    std::vector<std::pair<double, double>> nw(n);
    for (int i = 0; i < n; ++i) nw[i] = {J[i * n + i], mu0 * V[0 * n + i] * V[0 * n + i]};
    std::sort(nw.begin(), nw.end());
    for (int i = 0; i < n; ++i) { x[i] = nw[i].first; w[i] = nw[i].second; }
}

// ---------------------------------------------------------------------------
// Orthonormal Dubiner basis, evaluated in collapsed coordinates
//   a = (2 xi + eta - 1) / (1 - eta),  b = 2 eta - 1,
//   phi_pq = sqrt(2(2p+1)(p+q+1)) L_p(a) (1-eta)^p J_q^{(2p+1,0)}(b),
// with Jacobi polynomials from their explicit binomial sum and derivatives from
// d/dx J_n^{(al,be)} = (n+al+be+1)/2 J_{n-1}^{(al+1,be+1)}.
// ---------------------------------------------------------------------------
static double binom(double top, int k)
{
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r *= (top - k + i) / i;
    return r;
}

static double jacobi_sum(int n, double al, double be, double x)
{
    if (n < 0) return 0.0;
    double s = 0.0;
    const double u = 0.5 * (x - 1.0), v = 0.5 * (x + 1.0);
    for (int k = 0; k <= n; ++k) s += binom(n + al, n - k) * binom(n + be, k) * std::pow(u, k) * std::pow(v, n - k);
    return s;
}

static double jacobi_sum_d(int n, double al, double be, double x)
{
    return n == 0 ? 0.0 : 0.5 * (n + al + be + 1.0) * jacobi_sum(n - 1, al + 1.0, be + 1.0, x);
}

static void dubiner_at(int k, double xi, double eta, double* v, double* dxi, double* deta)
{
    const double om = 1.0 - eta;  // > 0 at every Gauss point
    const double a = (2.0 * xi + eta - 1.0) / om, b = 2.0 * eta - 1.0;
    int m = 0;
    for (int d = 0; d <= k; ++d)
        for (int q = 0; q <= d; ++q) {
            const int p = d - q;
            const double c = std::sqrt(2.0 * (2.0 * p + 1.0) * (p + q + 1.0));
            const double L = jacobi_sum(p, 0.0, 0.0, a), dL = jacobi_sum_d(p, 0.0, 0.0, a);
            const double J = jacobi_sum(q, 2.0 * p + 1.0, 0.0, b), dJ = jacobi_sum_d(q, 2.0 * p + 1.0, 0.0, b);
            const double omp = std::pow(om, p), omp1 = p >= 1 ? std::pow(om, p - 1) : 0.0;
            v[m] = c * L * omp * J;
            dxi[m] = c * 2.0 * dL * omp1 * J;
            deta[m] = c * ((dL * (1.0 + a) - p * L) * omp1 * J + L * omp * 2.0 * dJ);
            ++m;
        }
}

// Monomial basis xi^p eta^q, in the Dubiner order (d = p + q, then q = 0..d).
static void monomial_at(int k, double xi, double eta, double* v, double* dxi, double* deta)
{
    int m = 0;
    for (int d = 0; d <= k; ++d)
        for (int q = 0; q <= d; ++q) {
            const int p = d - q;
            const double xp = std::pow(xi, p), eq = std::pow(eta, q);
            v[m] = xp * eq;
            dxi[m] = p > 0 ? p * std::pow(xi, p - 1) * eq : 0.0;
            deta[m] = q > 0 ? q * xp * std::pow(eta, q - 1) : 0.0;
            ++m;
        }
}

static void basis_at(int k, int basis, double xi, double eta, double* v, double* dxi, double* deta)
{
    if (basis == DG_BASIS_MONOMIAL)
        monomial_at(k, xi, eta, v, dxi, deta);
    else
        dubiner_at(k, xi, eta, v, dxi, deta);
}

std::vector<double> build_tables(int k, int basis)
{
    const TabLayout T(k);
    std::vector<double> tab(T.size, 0.0);
    const int q = k + 2;
    double ga[16], gwa[16], gb[16], gwb[16];
    gauss_jacobi_gw(q, 0.0, 0.0, ga, gwa);
    gauss_jacobi_gw(q, 1.0, 0.0, gb, gwb);
    double v[32], dx[32], de[32];
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            const int g = i * q + j;
            const double xi = 0.25 * (1.0 + ga[i]) * (1.0 - gb[j]), eta = 0.5 * (1.0 + gb[j]);
            tab[T.vw + g] = 0.125 * gwa[i] * gwb[j];
            tab[T.vxi + g] = xi;
            tab[T.veta + g] = eta;
            basis_at(k, basis, xi, eta, v, dx, de);
            for (int m = 0; m < T.n; ++m) {
                tab[T.vphi + g * T.n + m] = v[m];
                tab[T.vdx + g * T.n + m] = dx[m];
                tab[T.vde + g * T.n + m] = de[m];
            }
        }
    for (int g = 0; g < q; ++g) {
        tab[T.et + g] = 0.5 * (1.0 + ga[g]);
        tab[T.ew + g] = 0.5 * gwa[g];
    }
    for (int l = 0; l < 3; ++l)
        for (int g = 0; g < q; ++g) {
            const double t = tab[T.et + g];
            double xi, eta;  // reference edge l runs from vertex l to vertex l+1
            if (l == 0) { xi = t; eta = 0.0; }
            else if (l == 1) { xi = 1.0 - t; eta = t; }
            else { xi = 0.0; eta = 1.0 - t; }
            basis_at(k, basis, xi, eta, v, dx, de);
            for (int m = 0; m < T.n; ++m) {
                tab[T.ephi + (l * q + g) * T.n + m] = v[m];
                tab[T.edx + (l * q + g) * T.n + m] = dx[m];
                tab[T.ede + (l * q + g) * T.n + m] = de[m];
            }
        }
    return tab;
}

std::vector<double> build_tensors(int k, const std::vector<double>& tab)
{
    const TabLayout L(k);
    const int n = L.n, nn = n * n, q = L.nqe;
    std::vector<double> ten((size_t)TenLayout::COUNT * nn, 0.0);
    auto at = [&](int t, int i, int j) -> double& { return ten[(size_t)t * nn + (size_t)j * n + i]; };
    for (int g = 0; g < L.nq; ++g) {
        const double w = tab[L.vw + g];
        const double* v = &tab[L.vphi + g * n];
        const double* dx = &tab[L.vdx + g * n];
        const double* de = &tab[L.vde + g * n];
        const double xi = tab[L.vxi + g], eta = tab[L.veta + g];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                at(TenLayout::VB + 0, i, j) += w * xi * v[i] * dx[j];
                at(TenLayout::VB + 1, i, j) += w * eta * v[i] * dx[j];
                at(TenLayout::VB + 2, i, j) += w * xi * v[i] * de[j];
                at(TenLayout::VB + 3, i, j) += w * eta * v[i] * de[j];
                at(TenLayout::VOL + 0, i, j) += w * dx[i] * dx[j];
                at(TenLayout::VOL + 1, i, j) += w * (dx[i] * de[j] + de[i] * dx[j]);
                at(TenLayout::VOL + 2, i, j) += w * de[i] * de[j];
                at(TenLayout::VOL + 3, i, j) += w * v[i] * dx[j];
                at(TenLayout::VOL + 4, i, j) += w * v[i] * de[j];
                at(TenLayout::VOL + 5, i, j) += w * v[i] * v[j];
            }
    }
    for (int l = 0; l < 3; ++l)
        for (int g = 0; g < q; ++g) {
            const double w = tab[L.ew + g], t = tab[L.et + g];
            const int ge = (l * q + g) * n;
            const double* v = &tab[L.ephi + ge];
            const double* dx = &tab[L.edx + ge];
            const double* de = &tab[L.ede + ge];
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) {
                    const int b = TenLayout::ED + 5 * l;
                    at(b + 0, i, j) += w * v[i] * v[j];
                    at(b + 1, i, j) += w * v[i] * dx[j];
                    at(b + 2, i, j) += w * v[i] * de[j];
                    at(b + 3, i, j) += w * dx[i] * v[j];
                    at(b + 4, i, j) += w * de[i] * v[j];
                    at(TenLayout::E1 + l, i, j) += w * t * v[i] * v[j];
                }
            // the neighbour's point: its edge lp at the reversed parameter (Gauss points are symmetric)
            for (int lp = 0; lp < 3; ++lp) {
                const int gl = (lp * q + (q - 1 - g)) * n;
                const double* u = &tab[L.ephi + gl];
                const double* ux = &tab[L.edx + gl];
                const double* ue = &tab[L.ede + gl];
                const int b = TenLayout::EO + 5 * (3 * l + lp);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) {
                        at(b + 0, i, j) += w * v[i] * u[j];
                        at(b + 1, i, j) += w * v[i] * ux[j];
                        at(b + 2, i, j) += w * v[i] * ue[j];
                        at(b + 3, i, j) += w * dx[i] * u[j];
                        at(b + 4, i, j) += w * de[i] * u[j];
                        at(TenLayout::F1 + 3 * l + lp, i, j) += w * t * v[i] * u[j];
                    }
            }
        }
    return ten;
}

std::vector<double> stage_tensors(int k, const std::vector<double>& ten, double kappa)
{
    const int n = (k + 1) * (k + 2) / 2, nn = n * n;
    std::vector<double> st((size_t)TenStage::COUNT * nn);
    for (int t = 0; t < 6; ++t)
        for (int e = 0; e < nn; ++e) st[(size_t)(TenStage::VOL + t) * nn + e] = ten[(size_t)(TenLayout::VOL + t) * nn + e];
    for (int l = 0; l < 3; ++l)
        for (int e = 0; e < nn; ++e) {
            const double* T = &ten[(size_t)(TenLayout::ED + 5 * l) * nn + e];  // E, DX, DY, TX, TY
            st[(size_t)(TenStage::ED + 3 * l) * nn + e] = T[0];
            st[(size_t)(TenStage::ED + 3 * l + 1) * nn + e] = kappa * T[3 * nn] - T[nn];
            st[(size_t)(TenStage::ED + 3 * l + 2) * nn + e] = kappa * T[4 * nn] - T[2 * nn];
        }
    auto copy = [&](int dst, int src, int cnt) {
        for (int t = 0; t < cnt; ++t)
            for (int e = 0; e < nn; ++e) st[(size_t)(dst + t) * nn + e] = ten[(size_t)(src + t) * nn + e];
    };
    copy(TenStage::EO, TenLayout::EO, 45);
    copy(TenStage::VB, TenLayout::VB, 4);
    copy(TenStage::E1, TenLayout::E1, 3);
    copy(TenStage::F1, TenLayout::F1, 9);
    return st;
}

std::vector<double> build_error_table(int k, int basis, int* nqr)
{
    const int q = k + 4, nq = q * q, n = (k + 1) * (k + 2) / 2;
    std::vector<double> t((size_t)nq * (3 + n));
    double ga[16], gwa[16], gb[16], gwb[16], v[32], dx[32], de[32];
    gauss_jacobi_gw(q, 0.0, 0.0, ga, gwa);
    gauss_jacobi_gw(q, 1.0, 0.0, gb, gwb);
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            const int g = i * q + j;
            const double xi = 0.25 * (1.0 + ga[i]) * (1.0 - gb[j]), eta = 0.5 * (1.0 + gb[j]);
            t[g] = 0.125 * gwa[i] * gwb[j];
            t[nq + g] = xi;
            t[2 * nq + g] = eta;
            basis_at(k, basis, xi, eta, v, dx, de);
            for (int m = 0; m < n; ++m) t[3 * nq + (size_t)g * n + m] = v[m];
        }
    *nqr = nq;
    return t;
}

static void free_device(dg_mesh* m)
{
    hipFree(m->d_xy); hipFree(m->d_nbr); hipFree(m->d_nbr_edge); hipFree(m->d_ebits); hipFree(m->d_row_ptr);
    hipFree(m->d_col_idx); hipFree(m->d_bnd_type); hipFree(m->d_bnd_el); hipFree(m->d_bnd_loc);
    hipFree(m->d_bnd_elems);
    hipFree(m->d_tab64); hipFree(m->d_tab32); hipFree(m->d_p1map); hipFree(m->d_ten64); hipFree(m->d_ten32);
    hipFree(m->d_tm64); hipFree(m->d_tm32); hipFree(m->d_tp64); hipFree(m->d_tp32); hipFree(m->d_mfcoef);
    hipFree(m->d_mref);
    hipFree(m->d_gt); hipFree(m->d_etab); hipFree(m->d_epart);
    hipFree(m->d_nodes); hipFree(m->d_elems); hipFree(m->d_eid); hipFree(m->d_owner);
    hipFree(m->d_dir); hipFree(m->d_neu); hipFree(m->d_dir_eid); hipFree(m->d_neu_eid);
}

template <typename T>
static int upload(T** dst, const std::vector<T>& src)
{
    size_t bytes = std::max<size_t>(src.size(), 1) * sizeof(T);
    if (hipMalloc((void**)dst, bytes) != hipSuccess) { *dst = nullptr; return DG_ERR_OOM; }
    if (!src.empty() && hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return DG_ERR_HIP;
    return DG_OK;
}

}  // namespace dg

using namespace dg;

extern "C" const char* dg_status_str(int32_t s)
{
    switch (s) {
    case DG_OK: return "DG_OK";
    case DG_NOT_CONVERGED: return "DG_NOT_CONVERGED";
    case DG_ERR_ARG: return "DG_ERR_ARG";
    case DG_ERR_ORIENTATION: return "DG_ERR_ORIENTATION";
    case DG_ERR_BOUNDARY: return "DG_ERR_BOUNDARY";
    case DG_ERR_NONMANIFOLD: return "DG_ERR_NONMANIFOLD";
    case DG_ERR_DEGREE: return "DG_ERR_DEGREE";
    case DG_ERR_METHOD: return "DG_ERR_METHOD";
    case DG_ERR_NONFINITE: return "DG_ERR_NONFINITE";
    case DG_ERR_HIP: return "DG_ERR_HIP";
    case DG_ERR_OOM: return "DG_ERR_OOM";
    }
    return "DG_UNKNOWN_STATUS";
}

extern "C" int32_t dg_default_penalty(int32_t method, int32_t degree, double* sigma, double* kappa)
{
    if (!sigma || !kappa) return DG_ERR_ARG;
    if (method != DG_NIPG && method != DG_SIPG && method != DG_IIPG) return DG_ERR_METHOD;
    if (degree < 0 || degree > DG_MAX_DEGREE) return DG_ERR_DEGREE;
    if (method == DG_NIPG) { *sigma = 1.0; *kappa = 1.0; return DG_OK; }
    if (degree == 0) return DG_ERR_DEGREE;  // 3k(k+1) = 0: no penalty
    *sigma = 3.0 * degree * (degree + 1);
    *kappa = method == DG_SIPG ? -1.0 : 0.0;
    return DG_OK;
}

namespace dg {
// Validates the section 2.1 arrays and fills the host-side mesh: connectivity,
// boundary classification, BSR pattern, per-element geometry and tables.
int build_host_mesh(const double* xy, int64_t n_nodes, const int32_t* elems, int64_t T, const int32_t* dir,
                    int64_t n_dir, const int32_t* neu, int64_t n_neu, int32_t degree, dg_mesh* m, bool with_tables)
{
    if (!xy || !elems || n_nodes <= 0 || T <= 0 || n_dir < 0 || n_neu < 0) return DG_ERR_ARG;
    if ((n_dir > 0 && !dir) || (n_neu > 0 && !neu)) return DG_ERR_ARG;
    if (degree < 0 || degree > DG_MAX_DEGREE) return DG_ERR_DEGREE;
    if (T > (int64_t)1 << 29) return DG_ERR_ARG;  // int32 block indices
    for (int64_t i = 0; i < 2 * n_nodes; ++i)
        if (!std::isfinite(xy[i])) return DG_ERR_NONFINITE;
    m->k = degree;
    const TabLayout L(degree);
    m->n = L.n; m->nq = L.nq; m->nqe = L.nqe;
    m->T = T; m->n_nodes = n_nodes;
    m->xy6.resize(6 * T);
    for (int64_t K = 0; K < T; ++K) {
        for (int l = 0; l < 3; ++l) {
            int32_t v = elems[3 * K + l];
            if (v < 0 || v >= n_nodes) return DG_ERR_ARG;
            m->xy6[6 * K + 2 * l] = xy[2 * v];
            m->xy6[6 * K + 2 * l + 1] = xy[2 * v + 1];
        }
        const double* p = &m->xy6[6 * K];
        double det = (p[2] - p[0]) * (p[5] - p[1]) - (p[4] - p[0]) * (p[3] - p[1]);
        if (!(det > 0.0)) return DG_ERR_ORIENTATION;
    }

    // Edge connectivity through a hash map keyed by the sorted node pair.
    auto key = [](int64_t a, int64_t b) -> uint64_t {
        uint64_t lo = (uint64_t)std::min(a, b), hi = (uint64_t)std::max(a, b);
        return (lo << 32) | hi;
    };
    std::unordered_map<uint64_t, int64_t> first;  // key -> 3K+l of the first half-edge
    first.reserve((size_t)(3 * T));
    m->nbr.assign(3 * T, INT32_MIN);
    m->nbr_edge.assign(T, 0);
    double hmax = 0.0;
    int64_t n_int = 0;
    for (int64_t K = 0; K < T; ++K)
        for (int l = 0; l < 3; ++l) {
            const int32_t a = elems[3 * K + l], b = elems[3 * K + (l + 1) % 3];
            const uint64_t kk = key(a, b);
            auto it = first.find(kk);
            if (it == first.end()) { first.emplace(kk, 3 * K + l); continue; }
            const int64_t h = it->second;
            if (h < 0) return DG_ERR_NONMANIFOLD;  // third element on this edge
            const int64_t K2 = h / 3;
            const int l2 = (int)(h % 3);
            // the two elements must traverse the shared edge in opposite directions
            if (K2 == K || elems[3 * K2 + l2] != b || elems[3 * K2 + (l2 + 1) % 3] != a) return DG_ERR_NONMANIFOLD;
            m->nbr[3 * K + l] = (int32_t)K2;
            m->nbr[3 * K2 + l2] = (int32_t)K;
            m->nbr_edge[K] |= l2 << (2 * l);
            m->nbr_edge[K2] |= l << (2 * l2);
            it->second = -1;
            ++n_int;
        }
    // Boundary classification: every unpaired half-edge must be listed once.
    std::unordered_map<uint64_t, int> bc;  // key -> 0 Dirichlet / 1 Neumann, +2 once used
    bc.reserve((size_t)(n_dir + n_neu));
    for (int64_t i = 0; i < n_dir + n_neu; ++i) {
        const int32_t* e = i < n_dir ? dir + 2 * i : neu + 2 * (i - n_dir);
        if (e[0] < 0 || e[0] >= n_nodes || e[1] < 0 || e[1] >= n_nodes) return DG_ERR_ARG;
        if (!bc.emplace(key(e[0], e[1]), i < n_dir ? 0 : 1).second) return DG_ERR_BOUNDARY;
    }
    m->n_dir = m->n_neu = 0;
    m->bnd_el.clear(); m->bnd_loc.clear(); m->bnd_type.clear();
    for (int64_t K = 0; K < T; ++K)
        for (int l = 0; l < 3; ++l) {
            const int32_t a = elems[3 * K + l], b = elems[3 * K + (l + 1) % 3];
            const double dx = xy[2 * b] - xy[2 * a], dy = xy[2 * b + 1] - xy[2 * a + 1];
            hmax = std::max(hmax, std::sqrt(dx * dx + dy * dy));
            if (m->nbr[3 * K + l] != INT32_MIN) continue;
            auto it = bc.find(key(a, b));
            if (it == bc.end() || it->second >= 2) return DG_ERR_BOUNDARY;
            const int type = it->second;
            it->second += 2;
            const int32_t bidx = (int32_t)m->bnd_el.size();
            m->nbr[3 * K + l] = -(bidx + 1);
            m->bnd_el.push_back((int32_t)K);
            m->bnd_loc.push_back(l);
            m->bnd_type.push_back(type);
            (type == 0 ? m->n_dir : m->n_neu)++;
        }
    for (auto& kv : bc)
        if (kv.second < 2) return DG_ERR_BOUNDARY;  // listed edge not on the boundary
    m->n_int = n_int;
    m->n_bnd = (int64_t)m->bnd_el.size();
    m->bnd_elems.clear();
    for (int32_t K : m->bnd_el)  // bnd_el is ascending
        if (m->bnd_elems.empty() || m->bnd_elems.back() != K) m->bnd_elems.push_back(K);
    m->hmax = hmax;

    // BSR pattern: block row K = [K, neighbours in local edge order].
    m->row_ptr.resize(T + 1);
    m->row_ptr[0] = 0;
    for (int64_t K = 0; K < T; ++K) {
        int c = 1;
        for (int l = 0; l < 3; ++l) c += m->nbr[3 * K + l] >= 0;
        m->row_ptr[K + 1] = m->row_ptr[K] + c;
    }
    m->nnzb = m->row_ptr[T];
    m->col_idx.resize(m->nnzb);
    for (int64_t K = 0; K < T; ++K) {
        int s = m->row_ptr[K];
        m->col_idx[s++] = (int32_t)K;
        for (int l = 0; l < 3; ++l)
            if (m->nbr[3 * K + l] >= 0) m->col_idx[s++] = m->nbr[3 * K + l];
    }
    if (with_tables) m->tab64 = build_tables(degree, m->basis);
    return DG_OK;
}
}  // namespace dg

extern "C" int32_t dg_mesh_create_basis(const double* xy, int64_t n_nodes, const int32_t* elems, int64_t T,
                                        const int32_t* dir, int64_t n_dir, const int32_t* neu, int64_t n_neu,
                                        int32_t degree, int32_t basis, dg_mesh** out)
{
    if (!out) return DG_ERR_ARG;
    *out = nullptr;
    if (basis != DG_BASIS_DUBINER && basis != DG_BASIS_MONOMIAL) return DG_ERR_ARG;
    dg_mesh* m = new (std::nothrow) dg_mesh();
    if (!m) return DG_ERR_OOM;
    m->basis = basis;
    int st = build_host_mesh(xy, n_nodes, elems, T, dir, n_dir, neu, n_neu, degree, m, true);
    if (st != DG_OK) { delete m; return st; }
    std::vector<float> tab32(m->tab64.begin(), m->tab64.end());
    if (hipGetDevice(&m->device) != hipSuccess) st = DG_ERR_HIP;
    if (st == DG_OK) st = upload(&m->d_xy, m->xy6);
    if (st == DG_OK) st = upload(&m->d_nbr, m->nbr);
    if (st == DG_OK) st = upload(&m->d_nbr_edge, m->nbr_edge);
    if (st == DG_OK) {
        // per element: neighbour edges (bits 2l, 2l+1), neighbour present (bit 8 + l),
        // Neumann boundary edge (bit 12 + l)
        std::vector<int32_t> eb((size_t)m->T);
        for (int64_t K = 0; K < m->T; ++K) {
            int32_t b = m->nbr_edge[K] & 63;
            for (int l = 0; l < 3; ++l) {
                const int32_t nb = m->nbr[3 * K + l];
                if (nb >= 0) b |= 1 << (8 + l);
                else if (m->bnd_type[-nb - 1] == 1) b |= 1 << (12 + l);
            }
            eb[K] = b;
        }
        st = upload(&m->d_ebits, eb);
    }
    if (st == DG_OK) st = upload(&m->d_row_ptr, m->row_ptr);
    if (st == DG_OK) st = upload(&m->d_col_idx, m->col_idx);
    if (st == DG_OK) st = upload(&m->d_bnd_type, m->bnd_type);
    if (st == DG_OK) st = upload(&m->d_bnd_el, m->bnd_el);
    if (st == DG_OK) st = upload(&m->d_bnd_loc, m->bnd_loc);
    if (st == DG_OK) st = upload(&m->d_bnd_elems, m->bnd_elems);
    if (st == DG_OK) st = upload(&m->d_tab64, m->tab64);
    if (st == DG_OK) st = upload(&m->d_tab32, tab32);
    if (st == DG_OK) st = upload(&m->d_etab, build_error_table(degree, basis, &m->nqr));
    if (st == DG_OK) st = upload(&m->d_epart, std::vector<double>(ERR_BLOCKS + 1, 0.0));
    if (st == DG_OK) {
        std::vector<double> gt((size_t)4 * m->T);
        for (int64_t K = 0; K < m->T; ++K) {
            const double* p = &m->xy6[6 * K];
            const double j11 = p[2] - p[0], j12 = p[4] - p[0], j21 = p[3] - p[1], j22 = p[5] - p[1];
            const double det = j11 * j22 - j12 * j21;
            gt[4 * K + 0] = j22 / det;   // G11
            gt[4 * K + 1] = -j12 / det;  // G21
            gt[4 * K + 2] = -j21 / det;  // G12
            gt[4 * K + 3] = j11 / det;   // G22
        }
        // per element and local edge l with a neighbour L: G_L^T (|e| n_K), the
        // neighbour's gradient map applied to the scaled outward normal of the
        // edge, |e| n = (dy, -dx) along the edge from vertex l to vertex l+1
        std::vector<double> mL((size_t)6 * m->T, 0.0);
        for (int64_t K = 0; K < m->T; ++K) {
            const double* p = &m->xy6[6 * K];
            const double j11 = p[2] - p[0], j12 = p[4] - p[0], j21 = p[3] - p[1], j22 = p[5] - p[1];
            const double evx[3] = {j11, j12 - j11, -j12}, evy[3] = {j21, j22 - j21, -j22};
            for (int l = 0; l < 3; ++l) {
                const int32_t L = m->nbr[3 * K + l];
                if (L < 0) continue;
                const double nx = evy[l], ny = -evx[l];
                const double* g = &gt[4 * (size_t)L];
                mL[6 * K + 2 * l] = g[0] * nx + g[1] * ny;
                mL[6 * K + 2 * l + 1] = g[2] * nx + g[3] * ny;
            }
        }
        st = upload(&m->d_gt, mL);
    }
    if (st == DG_OK && degree <= 3) {
        const std::vector<double> ref = build_tensors(degree, m->tab64);
        std::vector<double> ten;
        for (int kap = -1; kap <= 1; ++kap) {
            const std::vector<double> s = stage_tensors(degree, ref, (double)kap);
            ten.insert(ten.end(), s.begin(), s.end());
        }
        // each tensor as n columns (trial j) of values (test i), every column padded
        // with zeros to whole 16-byte words of the precision (the kernel's layout)
        const int n = (degree + 1) * (degree + 2) / 2;
        auto padded = [&](int per_word) {
            const int np = (n + per_word - 1) / per_word * per_word;
            const size_t nt = ten.size() / ((size_t)n * n);
            std::vector<double> out(nt * n * np, 0.0);
            for (size_t t = 0; t < nt; ++t)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) out[(t * n + j) * np + i] = ten[(t * n + j) * n + i];
            return out;
        };
        const std::vector<double> ten64 = padded(2);
        const std::vector<double> t32 = padded(4);
        const std::vector<float> ten32(t32.begin(), t32.end());
        st = upload(&m->d_ten64, ten64);
        if (st == DG_OK) st = upload(&m->d_ten32, ten32);
        if (st == DG_OK && degree >= 2) {
            // matrix-core sets: the staged tensors (trial-major) re-laid as rows in block order
            const int nn = n * n, nnp = MfmaSet::nnp(degree);
            std::vector<double> tm((size_t)3 * MfmaSet::COUNT * nnp, 0.0);
            auto put = [&](int ki, int row, int src) {  // src: TenStage index, or -1 for a zero row
                if (src < 0) return;
                const double* S = &ten[((size_t)ki * TenStage::COUNT + src) * nn];
                double* D = &tm[((size_t)ki * MfmaSet::COUNT + row) * nnp];
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < n; ++j) D[i * n + j] = S[j * n + i];
            };
            for (int ki = 0; ki < 3; ++ki) {
                for (int t = 0; t < 4; ++t) put(ki, t, TenStage::VOL + t);  // SXX SXY SYY CX
                put(ki, 4, TenStage::VOL + 4);                                // CY
                put(ki, 5, TenStage::VOL + 5);                                // MASS
                for (int t = 0; t < 4; ++t) put(ki, 6 + t, TenStage::VB + t);
                for (int l = 0; l < 3; ++l) {
                    for (int t = 0; t < 3; ++t) put(ki, 12 + 4 * l + t, TenStage::ED + 3 * l + t);
                    put(ki, 12 + 4 * l + 3, TenStage::E1 + l);
                }
                for (int c = 0; c < 9; ++c) {
                    const int base = MfmaSet::DIAG + MfmaSet::OFF * c;
                    for (int t = 0; t < 5; ++t) put(ki, base + t, TenStage::EO + 5 * c + t);
                    put(ki, base + 5, TenStage::F1 + c);
                }
            }
            // upwind point products from the edge tables (the same values the
            // point-by-point upwind sum multiplies)
            const TabLayout L(degree);
            const int Q = L.nqe;
            std::vector<double> tp((size_t)MfmaSet::PCOUNT * nnp, 0.0);
            auto ephi = [&](int l, int g, int i) { return m->tab64[L.ephi + (l * Q + g) * n + i]; };
            for (int l = 0; l < 3; ++l)
                for (int g = 0; g < Q; ++g) {
                    double* D = &tp[((size_t)l * MfmaSet::PTS + g) * nnp];
                    for (int i = 0; i < n; ++i)
                        for (int j = 0; j < n; ++j) D[i * n + j] = ephi(l, g, i) * ephi(l, g, j);
                }
            for (int l = 0; l < 3; ++l)
                for (int lp = 0; lp < 3; ++lp)
                    for (int g = 0; g < Q; ++g) {
                        double* D = &tp[((size_t)(3 + 3 * l + lp) * MfmaSet::PTS + g) * nnp];
                        for (int i = 0; i < n; ++i)
                            for (int j = 0; j < n; ++j) D[i * n + j] = ephi(l, g, i) * ephi(lp, Q - 1 - g, j);
                    }
            st = upload(&m->d_tm64, tm);
            if (st == DG_OK) st = upload(&m->d_tm32, std::vector<float>(tm.begin(), tm.end()));
            if (st == DG_OK) st = upload(&m->d_tp64, tp);
            if (st == DG_OK) st = upload(&m->d_tp32, std::vector<float>(tp.begin(), tp.end()));
        }
    }
    if (st == DG_OK) {
        // P[m][v]: coefficient of basis function m in the linear function with
        // vertex values u_v (k >= 1).  Orthonormal basis: int_ref lambda_v phi_m.
        // Monomials: lambda_1 = 1 - xi - eta, lambda_2 = xi, lambda_3 = eta.
        const TabLayout L(degree);
        std::vector<double> P(9, 0.0);
        if (basis == DG_BASIS_MONOMIAL) {
            if (degree >= 1) {
                const double Pm[9] = {1.0, 0.0, 0.0, -1.0, 1.0, 0.0, -1.0, 0.0, 1.0};
                P.assign(Pm, Pm + 9);
            }
        } else {
            for (int g = 0; g < L.nq && degree >= 1; ++g) {
                const double xi = m->tab64[L.vxi + g], eta = m->tab64[L.veta + g], w = m->tab64[L.vw + g];
                const double lam[3] = {1.0 - xi - eta, xi, eta};
                for (int mm = 0; mm < 3; ++mm)
                    for (int v = 0; v < 3; ++v) P[mm * 3 + v] += w * lam[v] * m->tab64[L.vphi + g * L.n + mm];
            }
        }
        st = upload(&m->d_p1map, P);
        m->phi0 = m->tab64[L.vphi];  // the constant function: sqrt 2 (Dubiner) or 1 (monomial)
        if (st == DG_OK && basis == DG_BASIS_MONOMIAL) {
            // reference Gram matrix int_ref phi_i phi_j (the volume rule is exact for it)
            std::vector<double> G((size_t)L.n * L.n, 0.0);
            for (int g = 0; g < L.nq; ++g)
                for (int i = 0; i < L.n; ++i)
                    for (int j = 0; j < L.n; ++j)
                        G[(size_t)i * L.n + j] +=
                            m->tab64[L.vw + g] * m->tab64[L.vphi + g * L.n + i] * m->tab64[L.vphi + g * L.n + j];
            st = upload(&m->d_mref, G);
        }
    }
    if (st == DG_OK) {
        // Edge ids for refinement: walking the elements in order and each
        // element's edges (v0 v1), (v1 v2), (v2 v0), an edge gets the next id
        // when it is met for the first time (a boundary edge, or an interior
        // edge whose other element comes later).
        std::vector<int32_t> eid(3 * T), owner(3 * T, 0);
        int32_t ne = 0;
        for (int64_t K = 0; K < T; ++K)
            for (int l = 0; l < 3; ++l) {
                const int32_t nb = m->nbr[3 * K + l];
                if (nb < 0 || nb > K) {
                    owner[3 * K + l] = 1;
                    eid[3 * K + l] = ne++;
                } else {
                    eid[3 * K + l] = eid[3 * (int64_t)nb + ((m->nbr_edge[K] >> (2 * l)) & 3)];
                }
            }
        m->n_edges = ne;
        // ids of the listed boundary edges, in the caller's order
        std::unordered_map<uint64_t, int32_t> bid;
        bid.reserve((size_t)m->n_bnd);
        for (int64_t i = 0; i < m->n_bnd; ++i) {
            const int64_t K = m->bnd_el[i];
            const int l = m->bnd_loc[i];
            const uint64_t a = (uint64_t)elems[3 * K + l], b = (uint64_t)elems[3 * K + (l + 1) % 3];
            bid.emplace((std::min(a, b) << 32) | std::max(a, b), eid[3 * K + l]);
        }
        auto ids = [&](const int32_t* e, int64_t cnt) {
            std::vector<int32_t> v((size_t)cnt);
            for (int64_t i = 0; i < cnt; ++i) {
                const uint64_t a = (uint64_t)e[2 * i], b = (uint64_t)e[2 * i + 1];
                v[i] = bid.at((std::min(a, b) << 32) | std::max(a, b));
            }
            return v;
        };
        st = upload(&m->d_nodes, std::vector<double>(xy, xy + 2 * n_nodes));
        if (st == DG_OK) st = upload(&m->d_elems, std::vector<int32_t>(elems, elems + 3 * T));
        if (st == DG_OK) st = upload(&m->d_eid, eid);
        if (st == DG_OK) st = upload(&m->d_owner, owner);
        if (st == DG_OK && n_dir > 0) st = upload(&m->d_dir, std::vector<int32_t>(dir, dir + 2 * n_dir));
        if (st == DG_OK && n_neu > 0) st = upload(&m->d_neu, std::vector<int32_t>(neu, neu + 2 * n_neu));
        if (st == DG_OK && n_dir > 0) st = upload(&m->d_dir_eid, ids(dir, n_dir));
        if (st == DG_OK && n_neu > 0) st = upload(&m->d_neu_eid, ids(neu, n_neu));
    }
    if (st != DG_OK) { free_device(m); delete m; return st; }
    *out = m;
    return DG_OK;
}

extern "C" int32_t dg_mesh_info_get(const dg_mesh* m, dg_mesh_info* out)
{
    if (!m || !out) return DG_ERR_ARG;
    out->n_elems = m->T;
    out->n_int_edges = m->n_int;
    out->n_dir_edges = m->n_dir;
    out->n_neu_edges = m->n_neu;
    out->nnzb = m->nnzb;
    out->n_dofs = m->T * m->n;
    out->degree = m->k;
    out->n_loc = m->n;
    out->n_q = m->nq;
    out->n_qe = m->nqe;
    out->basis = m->basis;
    out->reserved = 0;
    out->h_max = m->hmax;
    return DG_OK;
}

extern "C" int32_t dg_mesh_create(const double* xy, int64_t n_nodes, const int32_t* elems, int64_t T,
                                  const int32_t* dir, int64_t n_dir, const int32_t* neu, int64_t n_neu,
                                  int32_t degree, dg_mesh** out)
{
    return dg_mesh_create_basis(xy, n_nodes, elems, T, dir, n_dir, neu, n_neu, degree, DG_BASIS_DUBINER, out);
}

extern "C" void dg_mesh_destroy(dg_mesh* m)
{
    if (!m) return;
    free_device(m);
    delete m;
}

extern "C" int32_t dg_mesh_structure(const dg_mesh* m, int32_t* dev_row_ptr, int32_t* dev_col_idx, void* stream)
{
    if (!m || !dev_row_ptr || !dev_col_idx) return DG_ERR_ARG;
    hipStream_t s = (hipStream_t)stream;
    DG_HIP_CHECK(hipMemcpyAsync(dev_row_ptr, m->d_row_ptr, sizeof(int32_t) * (m->T + 1), hipMemcpyDeviceToDevice, s));
    DG_HIP_CHECK(hipMemcpyAsync(dev_col_idx, m->d_col_idx, sizeof(int32_t) * m->nnzb, hipMemcpyDeviceToDevice, s));
    return DG_OK;
}
