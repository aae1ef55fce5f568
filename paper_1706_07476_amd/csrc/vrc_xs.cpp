// Cross-section tables: validation, union energy grid and hashed log-energy
// index (host side, run once per vrc_set_xs_tables).
//
// Sec. 3 of the paper: the total cross section of every material is found
// for the ray energy by a hash-based lookup and linear interpolation between
// table values.  Here all materials are merged onto the union of their
// energy grids.  A material's piecewise-linear Sigma_t(E) (with its end
// values held outside its own table) is linear between consecutive union
// points, so interpolating on the union grid gives the same function; only
// the rounding of the inserted points differs.  One bracketing search per
// ray then serves every material, and the values of all materials at a grid
// point sit next to each other in memory.
#include <algorithm>
#include <cmath>
#include <limits>

#include "vrc_internal.h"

namespace vrc {

namespace {

// Sigma of one material's own table at energy x: linear between points,
// end values held outside (FP64).
double interp_own(const double *e, const double *s, int64_t K, double x)
{
    if (x <= e[0]) return s[0];
    if (x >= e[K - 1]) return s[K - 1];
    const double *p = std::upper_bound(e, e + K, x);
    int64_t k = (p - e) - 1;
    double slope = (s[k + 1] - s[k]) / (e[k + 1] - e[k]);
    return s[k] + slope * (x - e[k]);
}

template <typename R>
std::vector<int32_t> build_hash(const std::vector<R> &E, int M, float l2e0, float inv_dl2)
{
    const int K = static_cast<int>(E.size());
    std::vector<int32_t> hash(M);
    for (int b = 0; b < M; ++b) {
        double lower = std::exp2(static_cast<double>(l2e0) + static_cast<double>(b) / inv_dl2);
        R x = static_cast<R>(lower);
        int64_t k = (std::upper_bound(E.begin(), E.end(), x) - E.begin()) - 1;
        if (k < 0) k = 0;
        if (k > K - 2) k = std::max(K - 2, 0);
        hash[b] = static_cast<int32_t>(k);
    }
    return hash;
}

}  // namespace

vrc_status build_xs(int n_mat, const int64_t *offs, const double *energy, const double *sigma,
                    XsHost &out)
{
    if (n_mat < 1 || n_mat > kMaxMaterials)
        return set_error(VRC_ERR_INVALID, "n_mat must be in 1..64");
    if (!offs || !energy || !sigma) return set_error(VRC_ERR_INVALID, "null table pointer");
    if (offs[0] != 0) return set_error(VRC_ERR_INVALID, "offs[0] must be 0");
    std::vector<double> all;
    for (int m = 0; m < n_mat; ++m) {
        int64_t a = offs[m], b = offs[m + 1];
        if (b <= a) return set_error(VRC_ERR_INVALID, "every material needs at least one table point");
        if (b - a > (int64_t(1) << 30)) return set_error(VRC_ERR_INVALID, "table too large");
        for (int64_t i = a; i < b; ++i) {
            if (!(std::isfinite(energy[i]) && energy[i] > 0))
                return set_error(VRC_ERR_INVALID, "energies must be finite and positive");
            if (i > a && !(energy[i] > energy[i - 1]))
                return set_error(VRC_ERR_INVALID, "energies must be strictly increasing per material");
            if (!(std::isfinite(sigma[i]) && sigma[i] >= 0))
                return set_error(VRC_ERR_INVALID, "cross sections must be finite and >= 0");
            all.push_back(energy[i]);
        }
    }
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    if (all.size() > static_cast<size_t>(1) << 30) return set_error(VRC_ERR_INVALID, "union grid too large");

    XsHost x;
    x.set = true;
    x.n_mat = n_mat;
    x.K = static_cast<int>(all.size());
    x.E = all;
    x.S.resize(static_cast<size_t>(x.K) * n_mat);
    for (int m = 0; m < n_mat; ++m) {
        const double *e = energy + offs[m];
        const double *s = sigma + offs[m];
        int64_t Km = offs[m + 1] - offs[m];
        for (int k = 0; k < x.K; ++k) {
            // exact table values at the material's own points
            const double *p = std::lower_bound(e, e + Km, x.E[k]);
            double v = (p != e + Km && *p == x.E[k]) ? s[p - e] : interp_own(e, s, Km, x.E[k]);
            x.S[static_cast<size_t>(k) * n_mat + m] = v;
        }
    }
    x.s_stride32 = (n_mat + 3) / 4 * 4;
    x.s_stride64 = (n_mat + 1) / 2 * 2;

    // FP32 copy of the grid must stay strictly increasing to be usable
    std::vector<float> E32(x.K);
    x.f32_ok = true;
    for (int k = 0; k < x.K; ++k) {
        E32[k] = static_cast<float>(x.E[k]);
        if (!(std::isfinite(E32[k]) && E32[k] > 0)) x.f32_ok = false;
        if (k > 0 && !(E32[k] > E32[k - 1])) x.f32_ok = false;
    }

    // hash: M bins uniform in log2 E over the grid's range, about one to a
    // few grid points per bin, at most 8192 (32 KB of LDS)
    int M = 64;
    while (M < x.K && M < 8192) M *= 2;
    x.M = M;
    double l0 = std::log2(x.E.front());
    double l1 = std::log2(x.E.back());
    if (!(l1 > l0)) l1 = l0 + 1.0;
    x.l2e0 = static_cast<float>(l0);
    x.inv_dl2 = static_cast<float>(M / (l1 - l0));
    x.hash64 = build_hash<double>(x.E, M, x.l2e0, x.inv_dl2);
    if (x.f32_ok) x.hash32 = build_hash<float>(E32, M, x.l2e0, x.inv_dl2);
    else x.hash32 = x.hash64;
    out = std::move(x);
    return VRC_OK;
}

// Tables of mixtures of tabulated components: mixture k's Sigma is
// sum_j f_j Sigma_j(E) over its components.  Each component is piecewise
// linear with its end values held, so the sum is piecewise linear between
// consecutive points of the union of the components' grids: its values at
// those points (terms added in component order) describe it exactly up to
// rounding, and the mixture becomes an ordinary material table.
vrc_status mix_tables(int n_comp, const int64_t *comp_offs, const double *energy, const double *sigma, int n_mix,
                      const int64_t *mix_offs, const int32_t *mix_comp, const double *mix_frac,
                      std::vector<int64_t> &offs, std::vector<double> &e_out, std::vector<double> &s_out)
{
    if (n_comp < 1 || n_comp > (1 << 16)) return set_error(VRC_ERR_INVALID, "n_comp must be in 1..65536");
    if (n_mix < 1 || n_mix > kMaxMaterials) return set_error(VRC_ERR_INVALID, "n_mat must be in 1..64");
    if (!comp_offs || !energy || !sigma || !mix_offs || !mix_comp || !mix_frac)
        return set_error(VRC_ERR_INVALID, "null table or mixture pointer");
    if (comp_offs[0] != 0 || mix_offs[0] != 0) return set_error(VRC_ERR_INVALID, "offsets must start at 0");
    for (int c = 0; c < n_comp; ++c) {
        const int64_t a = comp_offs[c], b = comp_offs[c + 1];
        if (b <= a) return set_error(VRC_ERR_INVALID, "every component needs at least one table point");
        if (b - a > (int64_t(1) << 30)) return set_error(VRC_ERR_INVALID, "table too large");
        for (int64_t i = a; i < b; ++i) {
            if (!(std::isfinite(energy[i]) && energy[i] > 0))
                return set_error(VRC_ERR_INVALID, "energies must be finite and positive");
            if (i > a && !(energy[i] > energy[i - 1]))
                return set_error(VRC_ERR_INVALID, "energies must be strictly increasing per component");
            if (!(std::isfinite(sigma[i]) && sigma[i] >= 0))
                return set_error(VRC_ERR_INVALID, "cross sections must be finite and >= 0");
        }
    }
    offs.assign(1, 0);
    e_out.clear();
    s_out.clear();
    for (int k = 0; k < n_mix; ++k) {
        const int64_t a = mix_offs[k], b = mix_offs[k + 1];
        if (b <= a) return set_error(VRC_ERR_INVALID, "every mixture needs at least one component");
        if (b - a > 4096) return set_error(VRC_ERR_INVALID, "at most 4096 components per mixture");
        std::vector<double> grid;
        for (int64_t j = a; j < b; ++j) {
            const int c = mix_comp[j];
            if (c < 0 || c >= n_comp) return set_error(VRC_ERR_INVALID, "mixture names no such component");
            if (!(std::isfinite(mix_frac[j]) && mix_frac[j] >= 0))
                return set_error(VRC_ERR_INVALID, "mixture factors must be finite and >= 0");
            grid.insert(grid.end(), energy + comp_offs[c], energy + comp_offs[c + 1]);
        }
        std::sort(grid.begin(), grid.end());
        grid.erase(std::unique(grid.begin(), grid.end()), grid.end());
        if (e_out.size() + grid.size() > (static_cast<size_t>(1) << 30))
            return set_error(VRC_ERR_INVALID, "mixture tables too large");
        for (double x : grid) {
            double v = 0.0;
            for (int64_t j = a; j < b; ++j) {
                const int c = mix_comp[j];
                const double *e = energy + comp_offs[c];
                const double *sg = sigma + comp_offs[c];
                const int64_t K = comp_offs[c + 1] - comp_offs[c];
                const double *p = std::lower_bound(e, e + K, x);
                const double t = (p != e + K && *p == x) ? sg[p - e] : interp_own(e, sg, K, x);
                v += mix_frac[j] * t;
            }
            e_out.push_back(x);
            s_out.push_back(v);
        }
        offs.push_back(static_cast<int64_t>(e_out.size()));
    }
    return VRC_OK;
}

}  // namespace vrc
