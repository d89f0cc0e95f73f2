// Host runtime and C ABI of the Parareal-over-stencils library (gfx950).
//
// Responsibilities: argument validation and the stability guard (before any
// device work), tile layout of the stencil launches, descriptor tables,
// workspace layout, the Parareal orchestration of Algorithm 1 with all time
// slices of all instances batched on one device, optional HIP-graph replay,
// event timing, and the autotuner of the fused kernel variants.
#include "pr.h"
#include "pr_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using pr::ItemDesc;
using pr::PointItem;
using pr::VariantInfo;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(PR_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int g_fine_forced = 0, g_coarse_forced = 0;
int g_bpc_forced = 0;   // blocks-per-CU target forced while tuning (0: tuned or default)

// A kernel choice: fused variant and the launch-size target of the tile
// layout (blocks per CU, which sets the z-chunk depth; 0 = default).
struct Choice {
    int v = 0;
    int bpc = 0;
};
std::mutex g_tune_mu;
// (arch, which, nx, ny, nz, dtype, order, batch) -> choice of the tuner
using TuneKey = std::tuple<std::string, int, int, int, int, int, int, int>;
std::map<TuneKey, Choice> g_tuned;
bool g_cache_loaded = false;   // the PR_AUTOTUNE_CACHE file was read

// Architecture name of the current device ("gfx950"), or "none" without a
// device: tuned choices apply only on the architecture they were timed on.
const std::string &current_arch()
{
    static std::string arch;
    static std::once_flag once;
    std::call_once(once, [] {
        int n = 0, dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceCount(&n) == hipSuccess && n > 0 && hipGetDevice(&dev) == hipSuccess &&
            hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            arch = prop.gcnArchName;
            const size_t c = arch.find(':');
            if (c != std::string::npos) arch.resize(c);
        }
        if (arch.empty()) arch = "none";
    });
    return arch;
}

int load_tune_cache_locked(const char *path, int *loaded);

// Read the file named by PR_AUTOTUNE_CACHE once, before the first lookup.
void autoload_tune_cache_locked()
{
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char *path = std::getenv("PR_AUTOTUNE_CACHE");
    if (path && *path) {
        int n = 0;
        (void)load_tune_cache_locked(path, &n);
    }
}

// Tuned choice for a shape: the entry of this batch, else any batch of the shape.
bool tuned_choice(int which, const pr_problem &p, int dtype, int order, int batch, Choice *c)
{
    const std::string &arch = current_arch();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    autoload_tune_cache_locked();
    auto it = g_tuned.find({arch, which, p.n[0], p.n[1], p.n[2], dtype, order, batch});
    if (it == g_tuned.end()) {
        it = g_tuned.lower_bound({arch, which, p.n[0], p.n[1], p.n[2], dtype, order, 0});
        if (it == g_tuned.end()) return false;
        const auto &k = it->first;
        if (std::get<0>(k) != arch || std::get<1>(k) != which || std::get<2>(k) != p.n[0] ||
            std::get<3>(k) != p.n[1] || std::get<4>(k) != p.n[2] || std::get<5>(k) != dtype ||
            std::get<6>(k) != order)
            return false;
    }
    *c = it->second;
    return true;
}

void record_tuned(int which, const pr_problem &p, int dtype, int order, int batch, Choice c)
{
    const std::string &arch = current_arch();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    autoload_tune_cache_locked();
    g_tuned[{arch, which, p.n[0], p.n[1], p.n[2], dtype, order, batch}] = c;
}

int g_num_cus = 0;

int device_ready()
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(PR_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    if (g_num_cus == 0) {
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        g_num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    }
    return PR_OK;
}

// Maximum that keeps a NaN operand (std::max drops one in its second argument).
double nan_max(double m, double v) { return (v != v || v > m) ? v : m; }

size_t esize(int dtype) { return dtype == PR_FP64 ? 8 : 4; }
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t npts_of(const pr_problem &p) { return (int64_t)p.n[0] * p.n[1] * p.n[2]; }

// ---- validation -----------------------------------------------------------

int validate_problem(const pr_problem *p, bool need_parareal)
{
    if (!p) return fail(PR_EINVAL, "problem is NULL");
    const int minn = p->fine_order == 4 ? 5 : 3;
    for (int d = 0; d < 3; ++d) {
        if (p->n[d] < minn) return fail(PR_EINVAL, "n[%d] = %d < %d", d, p->n[d], minn);
        if (p->n[d] > 65536) return fail(PR_EINVAL, "n[%d] = %d too large", d, p->n[d]);
        if (!std::isfinite(p->a[d])) return fail(PR_EINVAL, "a[%d] not finite", d);
    }
    if (npts_of(*p) >= ((int64_t)1 << 31)) return fail(PR_EINVAL, "field of %lld points exceeds 2^31 - 1",
                                                       (long long)npts_of(*p));
    if (p->fine_order != 2 && p->fine_order != 4) return fail(PR_EINVAL, "fine_order must be 2 or 4");
    if (!(p->nu0 > 0.0) || !std::isfinite(p->nu0)) return fail(PR_EINVAL, "nu0 must be positive and finite");
    if (!std::isfinite(p->nu_amp) || !(std::fabs(p->nu_amp) < 1.0))
        return fail(PR_EINVAL, "|nu_amp| must be < 1 so that nu(t) > 0");
    if (!std::isfinite(p->nu_omega)) return fail(PR_EINVAL, "nu_omega not finite");
    if (!(p->T > 0.0) || !std::isfinite(p->T)) return fail(PR_EINVAL, "T must be positive and finite");
    if (p->nt_fine < 1 || p->nt_coarse < 1) return fail(PR_EINVAL, "step counts must be >= 1");
    if (need_parareal) {
        if (p->P < 1) return fail(PR_EINVAL, "P must be >= 1");
        if (p->nt_fine % p->P != 0) return fail(PR_EINVAL, "nt_fine = %d is not a multiple of P = %d", p->nt_fine, p->P);
        if (p->nt_coarse % p->P != 0)
            return fail(PR_EINVAL, "nt_coarse = %d is not a multiple of P = %d", p->nt_coarse, p->P);
        if (p->K < 0 || p->K > p->P) return fail(PR_EINVAL, "K = %d outside [0, P = %d]", p->K, p->P);
        if ((p->flags & PR_EARLY_STOP) && !(p->tol >= 0.0)) return fail(PR_EINVAL, "tol must be >= 0");
    }
    if (p->flags & ~(PR_NU_FROZEN | PR_ALLOW_UNSTABLE | PR_EARLY_STOP | PR_SKIP_CONVERGED | PR_COARSEN_G |
                     PR_CUBIC_INTERP))
        return fail(PR_EINVAL, "unknown flag bits 0x%x", p->flags);
    if ((p->flags & PR_CUBIC_INTERP) && !(p->flags & PR_COARSEN_G))
        return fail(PR_EINVAL, "PR_CUBIC_INTERP needs PR_COARSEN_G");
    if (p->flags & PR_COARSEN_G)
        for (int d = 0; d < 3; ++d)
            if (p->n[d] % 2 != 0 || p->n[d] / 2 < 3)
                return fail(PR_EINVAL, "PR_COARSEN_G needs even n[d] >= 6 (n[%d] = %d)", d, p->n[d]);
    return PR_OK;
}

// The grid G runs on: the problem's own, or with PR_COARSEN_G the grid
// coarsened by 2 per direction (same physics and time grid).
pr_problem coarse_grid(const pr_problem &p)
{
    pr_problem q = p;
    if (p.flags & PR_COARSEN_G) {
        for (int d = 0; d < 3; ++d) q.n[d] = p.n[d] / 2;
        q.flags &= ~(PR_COARSEN_G | PR_CUBIC_INTERP);
    }
    return q;
}

int interp_order(const pr_problem &p) { return (p.flags & PR_CUBIC_INTERP) ? 3 : 1; }

// ---- stability ------------------------------------------------------------

void margins(const pr_problem &p, double *fm, double *cm)
{
    const double numax = p.nu0 * (1.0 + std::fabs(p.nu_amp));
    const double numin = p.nu0 * (1.0 - std::fabs(p.nu_amp));
    double sa = 0.0, sd = 0.0;
    const pr_problem g = coarse_grid(p);   // G's grid
    for (int d = 0; d < 3; ++d) {
        sa += std::fabs(g.a[d]) * g.n[d];
        sd += (double)g.n[d] * g.n[d];
    }
    const double Dt = p.T / p.nt_coarse;
    *cm = Dt * (sa + 2.0 * numax * sd);

    const double dt = p.T / p.nt_fine;
    constexpr int NS = 48;
    double th[NS];
    for (int i = 0; i < NS; ++i) th[i] = M_PI * i / (NS - 1);
    // per-axis symbol parts: diffusion sd_d(theta) * n_d^2 and advection sa_d(theta) * n_d
    std::vector<double> D[3], A[3];
    for (int d = 0; d < 3; ++d) {
        D[d].resize(NS);
        A[d].resize(NS);
        const double n = p.n[d];
        for (int i = 0; i < NS; ++i) {
            const double t = th[i];
            if (p.fine_order == 4) {
                D[d][i] = (-2.0 * std::cos(2 * t) + 32.0 * std::cos(t) - 30.0) / 12.0 * n * n;
                A[d][i] = -p.a[d] * (8.0 * std::sin(t) - std::sin(2 * t)) / 6.0 * n;
            } else {
                D[d][i] = (2.0 * std::cos(t) - 2.0) * n * n;
                A[d][i] = -p.a[d] * std::sin(t) * n;
            }
        }
    }
    double worst = 0.0;
    const double nus[2] = {numin, numax};
    for (double nu : nus)
        for (int i = 0; i < NS; ++i)
            for (int j = 0; j < NS; ++j)
                for (int k = 0; k < NS; ++k) {
                    const std::complex<double> z(dt * nu * (D[0][i] + D[1][j] + D[2][k]),
                                                 dt * (A[0][i] + A[1][j] + A[2][k]));
                    const std::complex<double> R = 1.0 + z * (1.0 + z * (0.5 + z * (1.0 / 6.0 + z / 24.0)));
                    worst = std::max(worst, std::abs(R));
                }
    *fm = worst;
}

// Margins depend only on the grid, a, nu(t) bounds and step sizes; sweeps are
// called many times with the same problem, so results are memoised.
std::mutex g_margin_mu;
std::map<std::vector<double>, std::pair<double, double>> g_margin_cache;

void margins_cached(const pr_problem &p, double *fm, double *cm)
{
    const std::vector<double> key = {(double)p.n[0], (double)p.n[1], (double)p.n[2], p.a[0], p.a[1], p.a[2],
                                     p.nu0, p.nu_amp, p.T, (double)p.nt_fine, (double)p.nt_coarse,
                                     (double)p.fine_order, (double)(p.flags & PR_COARSEN_G)};
    {
        std::lock_guard<std::mutex> lk(g_margin_mu);
        auto it = g_margin_cache.find(key);
        if (it != g_margin_cache.end()) {
            *fm = it->second.first;
            *cm = it->second.second;
            return;
        }
    }
    margins(p, fm, cm);
    std::lock_guard<std::mutex> lk(g_margin_mu);
    if (g_margin_cache.size() > 4096) g_margin_cache.clear();
    g_margin_cache[key] = {*fm, *cm};
}

int stability_guard(const pr_problem &p, bool fine, bool coarse)
{
    if (p.flags & PR_ALLOW_UNSTABLE) return PR_OK;
    double fm = 0, cm = 0;
    margins_cached(p, &fm, &cm);
    if (fine && fm > 1.0 + 1e-12)
        return fail(PR_EUNSTABLE, "fine RK4 step unstable: max |R(dt mu)| = %.6g > 1", fm);
    if (coarse && cm > 1.0 + 1e-12)
        return fail(PR_EUNSTABLE,
                    "coarse Euler/upwind step unstable: Dt*(sum|a|/h + 2 nu_max sum 1/h^2) = %.6g > 1 "
                    "(raise nt_coarse or set PR_ALLOW_UNSTABLE)",
                    cm);
    return PR_OK;
}

// ---- variants and layout ---------------------------------------------------

int find_fine(const char *name)
{
    for (int v = 2; v < pr::fine_variant_count(); ++v)
        if (!std::strcmp(pr::fine_variant(v)->name, name)) return v;
    return -1;
}
int find_coarse(const char *name)
{
    for (int v = 2; v < pr::coarse_variant_count(); ++v)
        if (!std::strcmp(pr::coarse_variant(v)->name, name)) return v;
    return -1;
}

// ---- persisted autotune table ---------------------------------------------
//
// JSON written and read by the library only:
//   {"format": "pr-autotune-1", "entries": [
//     {"arch": "gfx950", "which": 0, "n": [128, 128, 128], "dtype": 2, "order": 2,
//      "batch": 16, "variant": "rk4w_f64_x128_y8_p2x1_w16", "blocks_per_cu": 0}, ...]}
// Variants are stored by name; entries naming a variant the library does not
// have are skipped when loading.

bool json_field(const std::string &obj, const char *key, size_t *pos)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t i = obj.find(k);
    if (i == std::string::npos) return false;
    i = obj.find(':', i + k.size());
    if (i == std::string::npos) return false;
    *pos = i + 1;
    return true;
}
bool json_int(const std::string &obj, const char *key, int *out)
{
    size_t i;
    if (!json_field(obj, key, &i)) return false;
    char *end = nullptr;
    const long v = std::strtol(obj.c_str() + i, &end, 10);
    if (end == obj.c_str() + i) return false;
    *out = (int)v;
    return true;
}
bool json_str(const std::string &obj, const char *key, std::string *out)
{
    size_t i;
    if (!json_field(obj, key, &i)) return false;
    const size_t a = obj.find('"', i);
    if (a == std::string::npos) return false;
    const size_t b = obj.find('"', a + 1);
    if (b == std::string::npos) return false;
    *out = obj.substr(a + 1, b - a - 1);
    return true;
}
bool json_int3(const std::string &obj, const char *key, int out[3])
{
    size_t i;
    if (!json_field(obj, key, &i)) return false;
    i = obj.find('[', i);
    if (i == std::string::npos) return false;
    const char *c = obj.c_str() + i + 1;
    for (int d = 0; d < 3; ++d) {
        char *end = nullptr;
        out[d] = (int)std::strtol(c, &end, 10);
        if (end == c) return false;
        c = end;
        while (*c == ' ' || *c == ',') ++c;
    }
    return true;
}

int load_tune_cache_locked(const char *path, int *loaded)
{
    *loaded = 0;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(PR_EINVAL, "cannot open autotune cache %s", path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    std::fclose(f);
    if (txt.find("\"pr-autotune-1\"") == std::string::npos)
        return fail(PR_EINVAL, "%s is not an autotune cache of this library", path);
    size_t i = txt.find("\"entries\"");
    if (i == std::string::npos) return fail(PR_EINVAL, "%s has no entries list", path);
    while ((i = txt.find('{', i)) != std::string::npos) {
        const size_t j = txt.find('}', i);
        if (j == std::string::npos) break;
        const std::string obj = txt.substr(i, j - i + 1);
        i = j + 1;
        std::string arch, name;
        int which, n[3], dtype, order, batch, bpc;
        if (!json_str(obj, "arch", &arch) || !json_int(obj, "which", &which) || !json_int3(obj, "n", n) ||
            !json_int(obj, "dtype", &dtype) || !json_int(obj, "order", &order) || !json_int(obj, "batch", &batch) ||
            !json_str(obj, "variant", &name) || !json_int(obj, "blocks_per_cu", &bpc))
            continue;
        if ((which != 0 && which != 1) || bpc < 0 || bpc > 64) continue;
        const int v = which == 0 ? find_fine(name.c_str()) : find_coarse(name.c_str());
        if (v < 2) continue;
        g_tuned[{arch, which, n[0], n[1], n[2], dtype, order, batch}] = Choice{v, bpc};
        ++*loaded;
    }
    return PR_OK;
}

int save_tune_cache_locked(const char *path)
{
    std::string out = "{\"format\": \"pr-autotune-1\", \"entries\": [";
    bool first = true;
    for (const auto &e : g_tuned) {
        const auto &k = e.first;
        const int which = std::get<1>(k), v = e.second.v;
        const VariantInfo *vi = which == 0 ? pr::fine_variant(v) : pr::coarse_variant(v);
        if (!vi) continue;
        char line[512];
        std::snprintf(line, sizeof line,
                      "%s\n  {\"arch\": \"%s\", \"which\": %d, \"n\": [%d, %d, %d], \"dtype\": %d, "
                      "\"order\": %d, \"batch\": %d, \"variant\": \"%s\", \"blocks_per_cu\": %d}",
                      first ? "" : ",", std::get<0>(k).c_str(), which, std::get<2>(k), std::get<3>(k),
                      std::get<4>(k), std::get<5>(k), std::get<6>(k), std::get<7>(k), vi->name, e.second.bpc);
        out += line;
        first = false;
    }
    out += "\n]}\n";
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(PR_EINVAL, "cannot write autotune cache %s", tmp.c_str());
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0)
        return fail(PR_EINVAL, "cannot write autotune cache %s", path);
    return PR_OK;
}

// After tuning: write the table to the file named by PR_AUTOTUNE_CACHE.
void save_tune_cache_env()
{
    const char *path = std::getenv("PR_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    (void)save_tune_cache_locked(path);
}

bool fine_applicable(int v, int dtype, int order, const pr_problem &p)
{
    if (v == 1) return true;
    const VariantInfo *vi = pr::fine_variant(v);
    return vi && vi->dtype == dtype && vi->order == order && p.n[0] % vi->nxp == 0 &&
           (vi->rowx == 0 || p.n[0] == vi->rowx);
}
bool coarse_applicable(int v, int dtype, const pr_problem &p)
{
    if (v == 1) return true;
    const VariantInfo *vi = pr::coarse_variant(v);
    return vi && vi->dtype == dtype && p.n[0] % vi->nxp == 0 && (vi->rowx == 0 || p.n[0] == vi->rowx);
}

// Points a fused RK4 kernel computes per output point of the grid's x-y
// plane, for a tile of tx x ty outputs with a halo of 4 per side.  A 2-D
// tiled kernel runs every stage on the whole tile.  An x-tiled row kernel
// (rowx == 0, one x tile per wavefront) runs a stage only in the wavefronts
// whose rows can still feed an output (stage s: rows s .. EY-1-s), so its y
// cost is the mean over the four stages of the rows of active wavefronts.
double fine_tile_cost(const VariantInfo *vi, bool xtiled, const pr_problem &p)
{
    const int nx = p.n[0], ny = p.n[1];
    const double wx = (double)((nx + vi->tx - 1) / vi->tx) * (vi->tx + 8) / nx;
    const int tiles_y = (ny + vi->ty - 1) / vi->ty;
    const int ey = vi->ty + 8;
    if (!xtiled) return wx * ((double)tiles_y * ey / ny);
    const int waves = vi->threads / 64, rows = ey / waves;
    double rs = 0;
    for (int s = 1; s <= 4; ++s)
        for (int w = 0; w < waves; ++w)
            if (w * rows + rows - 1 >= s && w * rows < ey - s) rs += rows;
    return wx * ((double)tiles_y * rs / 4 / ny);
}

// The candidate of one kernel family that computes the fewest points for
// the grid.
int cheapest_tile(const pr_problem &p, std::initializer_list<const char *> names, bool xtiled)
{
    int best_v = -1;
    double best = 1e300;
    for (const char *nm : names) {
        const int v = find_fine(nm);
        const VariantInfo *vi = pr::fine_variant(v);
        if (!vi || p.n[0] % vi->nxp) continue;
        const double c = fine_tile_cost(vi, xtiled, p);
        if (c < best * (1 - 1e-12)) {
            best = c;
            best_v = v;
        }
    }
    return best_v;
}

// Built-in choice (measured on the five workloads, on batches of the uneven
// workload's grid sizes, and on cubes of other sizes); batch = fields per
// launch.
int pick_fine_default(const pr_problem &p, int dtype, int batch)
{
    const int order = p.fine_order;
    const bool even = p.n[0] % 2 == 0;
    const char *name;
    if (dtype == PR_FP64) {
        // other widths: x-tiled rows (faster than the 2-D tiles on every
        // cube measured, n = 40 .. 384), the tile height that fits n_y best
        if (order == 2 && p.n[0] != 128 && p.n[0] != 64 && p.n[0] != 48 && p.n[0] != 32)
            return cheapest_tile(p, {"rk4x_f64_t56x8_p1x2_w8", "rk4x_f64_t56x16_p1x3_w8"}, true);
        name = order == 4 ? (p.n[0] == 128 ? "rk4h_f64_o4_x128_y8_p2_w16_d1"
                                             : "rk4hx_f64_o4_t120x8_p2_w16_d1")
               : p.n[0] == 128 ? "rk4w_f64_x128_y8_p2x1_w16"
               : p.n[0] == 64  ? (batch >= 4 ? "rk4w_f64_x64_y16_p1x2_w12" : "rk4w_f64_x64_y8_p1x2_w8")
               : p.n[0] == 48  ? "rk4s_f64_x48_y24_p3x1_w8"
                               : "rk4s_f64_x32_y32_p2x1_w10";
    } else if (order == 2 && p.n[0] == 64)
        name = batch >= 64 ? "rk4s_f32_x64_y24_p4x1_w8" : "rk4s_f32_x64_y40_p4x1_w12";
    else if (order == 2 && (p.n[0] == 96 || p.n[0] == 48 || p.n[0] == 32))
        name = p.n[0] == 96 ? "rk4s_f32_x96_y24_p6x1_w8"
               : p.n[0] == 48 ? "rk4s_f32_x48_y24_p3x1_w8"
                              : "rk4s_f32_x32_y32_p2x1_w10";
    else if (order == 2 && p.n[0] != 256 && p.n[0] != 128) {
        // n_x a multiple of 64: the 2-D tile (two x points per thread) that
        // computes the fewest points, whose 64-wide output tiles cover such
        // rows exactly (faster than x-tiled rows at 192 and 512, equal at 320
        // and 384); other widths: x-tiled rows (faster on every cube
        // measured, n = 40 .. 224)
        if (p.n[0] % 64 == 0)
            return cheapest_tile(p,
                                 {"rk4b_f32_t64x32_p2x2_d2", "rk4b_f32_t64x24_p2x2_d2", "rk4b_f32_t48x32_p2x2_d2",
                                  "rk4b_f32_t48x24_p2x2_d2"},
                                 false);
        name = "rk4x_f32_t56x40_p1x3_w16";
    } else
        name = order == 4 ? (p.n[0] == 128 ? "rk4h_f32_o4_x128_y8_p2_w16"
                             : even          ? "rk4r_f32_o4_t32x16_p2x2_d2"
                                             : "rk4_f32_o4_t32x16_p1x2")
               : p.n[0] == 256 ? "rk4w_f32_x256_y8_p4x2_w8"
                               : (batch >= 4 ? "rk4w_f32_x128_y16_p2x2_w12" : "rk4w_f32_x128_y8_p2x2_w8");
    return find_fine(name);
}

Choice pick_fine(const pr_problem &p, int dtype, int batch)
{
    Choice c;
    if (g_fine_forced) {
        c.v = g_fine_forced;
        c.bpc = g_bpc_forced;
        return c;
    }
    if (tuned_choice(0, p, dtype, p.fine_order, batch, &c)) return c;
    c.v = pick_fine_default(p, dtype, batch);
    return c;
}

// The coarse variant of a list that computes the fewest points for the
// grid (the x-tiled Euler rows skip steps per wavefront like the RK4 rows;
// S = 4 steps, halo 4).
int cheapest_coarse_rows(const pr_problem &p, std::initializer_list<const char *> names)
{
    int best_v = -1;
    double best = 1e300;
    for (const char *nm : names) {
        const int v = find_coarse(nm);
        const VariantInfo *vi = pr::coarse_variant(v);
        if (!vi) continue;
        const double c = fine_tile_cost(vi, true, p);
        if (c < best * (1 - 1e-12)) {
            best = c;
            best_v = v;
        }
    }
    return best_v;
}

// Built-in G for one grid: whole rows where a kernel exists; FP64 otherwise
// x-tiled rows (faster than the 2-D tiles on every cube measured, n = 40 ..
// 512) except on narrow rows; FP32 the 2-D tile where n_x is a multiple of
// 32 up to 128 (whose 32-wide tiles cover the row exactly: faster at 64 and
// 96), else x-tiled rows (faster at 40, 48, 100, 160, 200, 384, 512).
int pick_coarse_default(const pr_problem &p, int dtype)
{
    const int nx = p.n[0];
    if (dtype == PR_FP64) {
        if (nx == 128) return find_coarse("euler4w_f64_x128_y8_p2x1_w16");
        if (nx == 64) return find_coarse("euler4w_f64_x64_y8_p1x1_w16");
        // x-tiled rows unless their 64-column tiles compute far more points
        // than the 32-wide 2-D tiles (narrow rows such as 32): per computed
        // point they ran about a quarter faster
        const int xt = find_coarse("euler4x_f64_t56x24_p1x2_w16");
        const int tiled = find_coarse(nx % 2 == 0 ? "euler4b_f64_t32x32_p2x2_d2" : "euler4b_f64_t32x32_p1x4_d2");
        const VariantInfo *vx = pr::coarse_variant(xt), *vt = pr::coarse_variant(tiled);
        return 0.8 * fine_tile_cost(vx, true, p) <= fine_tile_cost(vt, false, p) ? xt : tiled;
    }
    if (nx == 256) return find_coarse("euler4w_f32_x256_y8_p4x1_w16");
    if (nx == 128) return find_coarse("euler4w_f32_x128_y8_p2x1_w16");
    if (nx % 32 == 0 && nx < 128) return find_coarse("euler4b_f32_t32x32_p2x2_d2");
    // three rows per wavefront (more work per barrier) beyond 64 rows; on
    // shorter grids the tile height that fits n_y best
    if (p.n[1] > 64) return find_coarse("euler4x_f32_t56x40_p1x3_w16");
    return cheapest_coarse_rows(p, {"euler4x_f32_t56x24_p1x2_w16", "euler4x_f32_t56x40_p1x3_w16"});
}

// Built-in G for instances of different widths in one plan (one launch per
// slice boundary covers all of them): FP32 on even widths the 2-D tile
// (measured best on the uneven batch of 48..128 cubes: chain 84 ms against
// 90-107 ms for x-tiled rows), otherwise x-tiled rows.
int pick_coarse_mixed(int dtype, bool all_even)
{
    if (dtype == PR_FP64) return find_coarse("euler4x_f64_t56x24_p1x2_w16");
    return find_coarse(all_even ? "euler4b_f32_t32x32_p2x2_d2" : "euler4x_f32_t56x40_p1x3_w16");
}

Choice pick_coarse(const pr_problem &p, int dtype, int batch)
{
    Choice c;
    if (g_coarse_forced) {
        c.v = g_coarse_forced;
        c.bpc = g_bpc_forced;
        return c;
    }
    if (tuned_choice(1, p, dtype, 0, batch, &c)) return c;
    c.v = pick_coarse_default(p, dtype);
    return c;
}

constexpr int kRefThreads = 256;

// Fill geometry, physics and tile layout of one sweep item (not pointers).
void fill_item(ItemDesc &it, const pr_problem &p, bool fine)
{
    it.nx = p.n[0];
    it.ny = p.n[1];
    it.nz = p.n[2];
    it.dt = fine ? p.T / p.nt_fine : p.T / p.nt_coarse;
    it.nu0 = p.nu0;
    it.nu_amp = p.nu_amp;
    it.nu_omega = p.nu_omega;
    for (int d = 0; d < 3; ++d) {
        it.inv_h2[d] = (double)p.n[d] * p.n[d];
        it.a_over_h[d] = p.a[d] * p.n[d];
    }
    it.frozen = (fine && (p.flags & PR_NU_FROZEN)) ? 1 : 0;
}

// Tile layout of a launch: tiles per item, z chunks and block ranges
// (assigned in item order); returns the total number of blocks.  Chunks are
// at least zmin planes deep; a block walks its chunk plus `fill` planes of
// pipeline fill.  occ = resident blocks per compute unit of the variant;
// bpc = resident blocks per compute unit to assume instead (0: occ).
int layout(std::vector<ItemDesc> &items, const VariantInfo *vi, bool ref, int zmin, int fill, int bpc, int occ)
{
    const int cus = std::max(g_num_cus, 1);
    const int64_t cap = (int64_t)(bpc > 0 ? bpc : std::max(occ, 1)) * cus;
    if (ref) {
        int b = 0;
        for (auto &it : items) {
            const int64_t n = (int64_t)it.nx * it.ny * it.nz;
            it.tiles_x = it.tiles_y = it.zchunks = 1;
            it.tz = it.nz;
            it.nblocks = (int)((n + kRefThreads - 1) / kRefThreads);
            it.block_begin = b;
            b += it.nblocks;
        }
        return b;
    }
    int64_t bxy = 0;
    int nzmax = 1;
    for (auto &it : items) {
        it.tiles_x = (it.nx + vi->tx - 1) / vi->tx;
        it.tiles_y = (it.ny + vi->ty - 1) / vi->ty;
        bxy += (int64_t)it.tiles_x * it.tiles_y;
        nzmax = std::max(nzmax, it.nz);
    }
    // The launch runs in rounds of `cap` resident blocks, each taking time in
    // proportion to the planes it walks.  Take the chunk count with the
    // fewest rounds x planes per block: enough chunks to fill the device, and
    // no last, mostly empty round of long blocks.
    int want = 1;
    int64_t best = INT64_MAX;
    const int zcmax = std::max(1, nzmax / zmin);
    for (int zc = 1; zc <= zcmax; ++zc) {
        const int tz = (nzmax + zc - 1) / zc;
        if ((nzmax + tz - 1) / tz != zc) continue;   // the layout of a smaller count
        const int64_t rounds = (bxy * zc + cap - 1) / cap;
        const int64_t cost = rounds * (tz + fill);
        if (cost < best) {
            best = cost;
            want = zc;
        }
    }
    int b = 0;
    for (auto &it : items) {
        const int maxz = std::max(1, it.nz / zmin);
        const int zc = std::min(want, maxz);
        it.tz = (it.nz + zc - 1) / zc;
        it.zchunks = (it.nz + it.tz - 1) / it.tz;
        it.nblocks = it.tiles_x * it.tiles_y * it.zchunks;
        it.block_begin = b;
        b += it.nblocks;
    }
    return b;
}

const VariantInfo *fine_info(int v) { return v >= 2 ? pr::fine_variant(v) : nullptr; }
const VariantInfo *coarse_info(int v) { return v >= 2 ? pr::coarse_variant(v) : nullptr; }
int coarse_steps_per_launch(int v) { return v >= 2 ? pr::coarse_variant(v)->steps : 1; }

// ---- sweeps -----------------------------------------------------------------

// Scratch fields per item (3 per field of the batch) are reserved for the
// unfused reference kernels and for every fourth-order problem, whose fine
// variants may take two launches per step through them.
bool scratch_reserved(const pr_problem &p, bool fine_ref) { return fine_ref || p.fine_order == 4; }

size_t sweep_ws(const pr_problem &p, int dtype, int batch, bool fine_ref)
{
    const size_t states = (size_t)batch * npts_of(p) * esize(dtype);
    return align256((size_t)batch * sizeof(ItemDesc)) + align256(states) +
           (scratch_reserved(p, fine_ref) ? 3 * align256(states) : 0);
}

int sweep_common(const pr_problem *prob_in, int dtype, int batch, const void *u_in, void *u_out,
                 const int64_t *step0, int nsteps, void *ws, size_t ws_bytes, void *stream, bool fine)
{
    int rc = validate_problem(prob_in, false);
    if (rc) return rc;
    // a sweep runs on the grid it is given: the plan-level coarsening flags do not apply
    pr_problem local = *prob_in;
    local.flags &= ~(PR_COARSEN_G | PR_CUBIC_INTERP);
    const pr_problem *prob = &local;
    if (dtype != PR_FP32 && dtype != PR_FP64) return fail(PR_EINVAL, "dtype must be PR_FP32 or PR_FP64");
    if (batch < 1) return fail(PR_EINVAL, "batch must be >= 1");
    if (nsteps < 0) return fail(PR_EINVAL, "nsteps must be >= 0");
    if (!u_in || !u_out) return fail(PR_EINVAL, "u_in/u_out is NULL");
    if (!step0) return fail(PR_EINVAL, "step0 is NULL");
    for (int b = 0; b < batch; ++b)
        if (step0[b] < 0) return fail(PR_EINVAL, "step0[%d] < 0", b);
    const size_t bytes = (size_t)batch * npts_of(*prob) * esize(dtype);
    const char *a = (const char *)u_in, *o = (const char *)u_out;
    if (((uintptr_t)a | (uintptr_t)o) & 15) return fail(PR_EINVAL, "u_in/u_out must be 16-byte aligned");
    if (a < o + bytes && o < a + bytes) return fail(PR_EINVAL, "u_in and u_out overlap");
    rc = stability_guard(*prob, fine, !fine);
    if (rc) return rc;
    const Choice ch = fine ? pick_fine(*prob, dtype, batch) : pick_coarse(*prob, dtype, batch);
    const int v = ch.v;
    if (v < 1) return fail(PR_EUNSUPPORTED, "no kernel variant for this problem");
    if (fine ? !fine_applicable(v, dtype, prob->fine_order, *prob) : !coarse_applicable(v, dtype, *prob))
        return fail(PR_EUNSUPPORTED, "selected kernel variant %d does not apply to this dtype/order/n_x", v);
    const bool ref = (v == 1);
    const size_t need = sweep_ws(*prob, dtype, batch, fine && ref);
    if (!ws || ws_bytes < need) return fail(PR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    rc = device_ready();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (nsteps == 0) {
        HIPCHK(hipMemcpyAsync(u_out, u_in, bytes, hipMemcpyDeviceToDevice, s));
        return PR_OK;
    }
    char *w = (char *)ws;
    ItemDesc *table = (ItemDesc *)w;
    char *tmp = w + align256((size_t)batch * sizeof(ItemDesc));
    char *scr = tmp + align256(bytes);
    const size_t fb = (size_t)npts_of(*prob) * esize(dtype);
    std::vector<ItemDesc> items(batch);
    for (int b = 0; b < batch; ++b) {
        ItemDesc &it = items[b];
        std::memset(&it, 0, sizeof it);
        fill_item(it, *prob, fine);
        it.src0 = a + b * fb;
        it.dst = (char *)u_out + b * fb;
        it.tmp = tmp + b * fb;
        it.scratch = scr + 3 * b * fb;
        it.step0 = step0[b];
        it.nsteps = nsteps;
    }
    const VariantInfo *vi = fine ? fine_info(v) : coarse_info(v);
    const int zmin = 2;
    const int fill = fine ? 8 : 2 * coarse_steps_per_launch(v);
    const int occ = fine ? pr::fine_occupancy(v) : pr::coarse_occupancy(v);
    const int nblocks = layout(items, vi, ref, zmin, fill, ch.bpc, occ);
    HIPCHK(pr::launch_write_items(items.data(), batch, table, s));
    if (fine) {
        for (int j = 0; j < nsteps; ++j)
            HIPCHK(pr::launch_fine_step(v, dtype, prob->fine_order, table, batch, nblocks, j, s));
    } else {
        const int S = coarse_steps_per_launch(v);
        const int nch = (nsteps + S - 1) / S;
        for (int c = 0; c < nch; ++c) HIPCHK(pr::launch_coarse_chunk(v, dtype, table, batch, nblocks, c, s));
    }
    return PR_OK;
}

}  // namespace

// ===========================================================================
// Plans
// ===========================================================================

struct pr_plan {
    int ninst = 0;
    int mode = 0;
    int dtype = PR_FP64;  // sweep dtype
    int K = 0;
    uint32_t flags = 0;
    int coarse_v = 0;
    int coarse_bpc = 0;   // blocks-per-CU target of the coarse layout (0: default)
    bool mixed = false, per_slice = false, graph = false, timed = false, skip = false, early = false;
    std::vector<pr_problem> probs;
    int Pmax = 0;

    struct Inst {
        int64_t npts;
        int P, nf, nc;
        double *U;                 // (P+1) FP64 states
        char *Ulo;                 // (P+1) sweep states (== U in FP64 mode)
        char *Fv, *Ftmp, *Gold[2], *Gtmp, *Fscr;
        char *Cin, *Cout, *Ctmp;   // coarsened G: restricted input, coarse result, ping-pong (npts/8 each)
        double *part;              // P x kNormBlocks x 4 correction partials
        double *refpart;           // kNormBlocks x 4
    };
    std::vector<Inst> inst;

    // F launch groups: instances that share a fused variant and layout.  Each
    // group is one launch per fine step; groups hold disjoint instances.
    struct FineGroup {
        int v = 0, bpc = 0;                      // variant, blocks-per-CU target (0: default)
        std::vector<int> insts;                  // instance indices
        std::vector<int> off, cnt;               // per k: offset into fine_tab, items
        std::vector<std::vector<int>> active;    // per k, per step j: blocks of the active prefix
    };
    std::vector<FineGroup> fgroups;
    std::vector<int> inst_group;        // instance -> group
    // groups 1.. run on their own streams, forked from and joined back to
    // the solve's stream around every F phase (the groups' instances are
    // disjoint, so their launches may overlap)
    std::vector<hipStream_t> aux;
    hipEvent_t fork_ev = nullptr;
    std::vector<hipEvent_t> join_ev;

    // Pipelined schedule (PR_MODE_PIPELINED): slices [pg_begin[g],
    // pg_begin[g+1]) form slice group g.  F of (k, g) runs, group by group, on
    // fstream[f] for each launch group f (table ptab[(k*npg + g)*nfg + f]);
    // events: ready[k*npg + g] (on the solve's stream: F of (k, g) may start),
    // first[..] and done[..] (on the F streams, per table: its first step,
    // which reads U^k_n, has run; all its steps have run), and per table the
    // timing pair tbeg/tend (PR_MODE_TIMED only).
    bool pipe = false;
    int npg = 0;
    std::vector<int> pg_begin;
    struct PipeTab {
        int off = 0, cnt = 0;
        std::vector<int> active;
    };
    std::vector<PipeTab> ptab;
    std::vector<hipStream_t> fstream;
    std::vector<hipEvent_t> ready, first, done, tbeg, tend;

    // device tables
    ItemDesc *fine_tab = nullptr;       // per k and group: the group's items (batched layout)
    ItemDesc *slice_tab = nullptr;      // per-slice layout: all (i, n), block_begin = 0
    std::vector<int> slice_index;       // (i, n) -> index into slice_tab
    std::vector<int> slice_blocks;      // blocks of each slice_tab item
    std::vector<int> slice_var;         // fine variant of each slice_tab item
    ItemDesc *coarse_tab = nullptr;     // [parity][n] -> up to ninst items
    bool coarsen = false;               // PR_COARSEN_G: G = prolong(coarse sweep(restrict(U)))
    int iorder = 1;                     // interpolation order of the coarsened G
    ItemDesc *rst_tab = nullptr;        // [n][ninst] restriction U_n -> Cin
    ItemDesc *pro_tab = nullptr;        // [parity][n][ninst] interpolation Cout -> Gold[parity]_n
    std::vector<int> coarse_cnt;        // per n: items (instances with P_i > n)
    std::vector<int> coarse_blocks;     // per (parity, n)
    std::vector<int> coarse_nch;        // per n: chunks of the longest item
    PointItem *pt_assign = nullptr;     // [n][ninst]   init: U_{n+1} = Gold0_n
    PointItem *pt_corr = nullptr;       // [parity][n][ninst]
    PointItem *pt_skip = nullptr;       // [parity][n][ninst] b = c = Gold[parity]
    PointItem *pt_final = nullptr;      // [k][sum P_i] per-slice finals
    PointItem *io_u0 = nullptr;         // [ninst] written per solve
    PointItem *io_uT = nullptr;         // [ninst]
    PointItem *io_ref = nullptr;        // [K][ninst] partials + final
    double *dlog = nullptr;             // [K][sum P_i][4]
    double *dlog_ref = nullptr;         // [K][ninst][4]
    std::vector<int> slice_base;        // per instance: offset of its slices in sum P_i
    int sumP = 0;

    hipStream_t own = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph_h = nullptr;
    std::vector<hipEvent_t> ev;
    int iters_done = 0;
    double timings[6] = {0, 0, 0, 0, 0, 0};
    bool had_ref_graph = false;
};

namespace {

struct Layout {
    size_t total = 0;
};

// Lay out (or only size) the plan workspace.  With plan == nullptr only the
// size is computed.
size_t plan_layout(const pr_problem *probs, int ninst, int mode, char *base, pr_plan *plan)
{
    const bool mixed = (mode & 1) != 0;
    const int dtype = mixed ? PR_FP32 : PR_FP64;
    const size_t es = esize(dtype);
    const bool fine_ref = (g_fine_forced == 1);
    const int K = probs[0].K;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    int sumP = 0, Pmax = 0;
    for (int i = 0; i < ninst; ++i) {
        sumP += probs[i].P;
        Pmax = std::max(Pmax, probs[i].P);
    }
    for (int i = 0; i < ninst; ++i) {
        const pr_problem &p = probs[i];
        const size_t n = (size_t)npts_of(p);
        pr_plan::Inst in{};
        in.npts = (int64_t)n;
        in.P = p.P;
        in.nf = p.nt_fine / p.P;
        in.nc = p.nt_coarse / p.P;
        in.U = (double *)take((p.P + 1) * n * 8);
        in.Ulo = mixed ? take((p.P + 1) * n * es) : (char *)in.U;
        in.Fv = take(p.P * n * es);
        in.Ftmp = take(p.P * n * es);
        in.Gold[0] = take(p.P * n * es);
        in.Gold[1] = take(p.P * n * es);
        in.Gtmp = take(n * es);
        in.Fscr = scratch_reserved(p, fine_ref) ? take(3 * p.P * n * es) : nullptr;
        const bool crs = (p.flags & PR_COARSEN_G) != 0;
        in.Cin = crs ? take(n / 8 * es) : nullptr;
        in.Cout = crs ? take(n / 8 * es) : nullptr;
        in.Ctmp = crs ? take(n / 8 * es) : nullptr;
        in.part = (double *)take((size_t)p.P * pr::kNormBlocks * 4 * 8);
        in.refpart = (double *)take((size_t)pr::kNormBlocks * 4 * 8);
        if (plan) plan->inst.push_back(in);
    }
    const int Kt = std::max(K, 1);
    // the pipelined schedule keeps a second set of F tables, cut by slice group
    const size_t fine_sets = (mode & PR_MODE_PIPELINED) ? 2 : 1;
    char *fine_tab = take(fine_sets * Kt * sumP * sizeof(ItemDesc));
    char *slice_tab = take((size_t)sumP * sizeof(ItemDesc));
    char *coarse_tab = take((size_t)2 * Pmax * ninst * sizeof(ItemDesc));
    char *rst_tab = take((size_t)Pmax * ninst * sizeof(ItemDesc));
    char *pro_tab = take((size_t)2 * Pmax * ninst * sizeof(ItemDesc));
    char *pt_assign = take((size_t)Pmax * ninst * sizeof(PointItem));
    char *pt_corr = take((size_t)2 * Pmax * ninst * sizeof(PointItem));
    char *pt_skip = take((size_t)2 * Pmax * ninst * sizeof(PointItem));
    char *pt_final = take((size_t)Kt * sumP * sizeof(PointItem));
    char *io_u0 = take((size_t)ninst * sizeof(PointItem));
    char *io_uT = take((size_t)ninst * sizeof(PointItem));
    char *io_ref = take((size_t)Kt * ninst * sizeof(PointItem));
    char *dlog = take((size_t)Kt * sumP * 4 * 8);
    char *dlog_ref = take((size_t)Kt * ninst * 4 * 8);
    if (plan) {
        plan->fine_tab = (ItemDesc *)fine_tab;
        plan->slice_tab = (ItemDesc *)slice_tab;
        plan->coarse_tab = (ItemDesc *)coarse_tab;
        plan->rst_tab = (ItemDesc *)rst_tab;
        plan->pro_tab = (ItemDesc *)pro_tab;
        plan->pt_assign = (PointItem *)pt_assign;
        plan->pt_corr = (PointItem *)pt_corr;
        plan->pt_skip = (PointItem *)pt_skip;
        plan->pt_final = (PointItem *)pt_final;
        plan->io_u0 = (PointItem *)io_u0;
        plan->io_uT = (PointItem *)io_uT;
        plan->io_ref = (PointItem *)io_ref;
        plan->dlog = (double *)dlog;
        plan->dlog_ref = (double *)dlog_ref;
        plan->sumP = sumP;
        plan->Pmax = Pmax;
    }
    return off;
}

int validate_plan_args(const pr_problem *probs, int ninst, int mode)
{
    if (!probs) return fail(PR_EINVAL, "probs is NULL");
    if (ninst < 1) return fail(PR_EINVAL, "ninst must be >= 1");
    if (mode & ~(PR_MODE_MIXED | PR_MODE_PER_SLICE | PR_MODE_GRAPH | PR_MODE_TIMED | PR_MODE_PIPELINED |
                 PR_MODE_PIPELINE_GROUPS(255)))
        return fail(PR_EINVAL, "unknown mode bits 0x%x", mode);
    if ((mode & PR_MODE_PIPELINE_GROUPS(255)) && !(mode & PR_MODE_PIPELINED))
        return fail(PR_EINVAL, "slice groups given without PR_MODE_PIPELINED");
    if ((mode & PR_MODE_PIPELINED) && (mode & PR_MODE_PER_SLICE))
        return fail(PR_EINVAL, "PR_MODE_PIPELINED does not combine with PR_MODE_PER_SLICE");
    if ((mode & PR_MODE_PIPELINED) && (probs[0].flags & PR_EARLY_STOP))
        return fail(PR_EINVAL, "PR_MODE_PIPELINED does not combine with PR_EARLY_STOP (the norms of iteration k "
                               "are read on the host before F of iteration k+1 may start)");
    for (int i = 0; i < ninst; ++i) {
        int rc = validate_problem(&probs[i], true);
        if (rc) {
            g_err = "instance " + std::to_string(i) + ": " + g_err;
            return rc;
        }
        if (probs[i].K != probs[0].K) return fail(PR_EINVAL, "K differs between instances");
        if (probs[i].flags != probs[0].flags) return fail(PR_EINVAL, "flags differ between instances");
        if (probs[i].tol != probs[0].tol) return fail(PR_EINVAL, "tol differs between instances");
        rc = stability_guard(probs[i], true, true);
        if (rc) {
            g_err = "instance " + std::to_string(i) + ": " + g_err;
            return rc;
        }
    }
    return PR_OK;
}

template <typename T>
int upload(T *dev, const std::vector<T> &host)
{
    if (host.empty()) return PR_OK;
    HIPCHK(hipMemcpy(dev, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
    return PR_OK;
}

char *slice_ptr(char *base, int n, int64_t npts, size_t es) { return base + (size_t)n * npts * es; }

// The F group with the most fine LUPs per solve (the plan's dominant launch).
int primary_group(const pr_plan *pl)
{
    int best = 0;
    double most = -1;
    for (int g = 0; g < (int)pl->fgroups.size(); ++g) {
        double w = 0;
        for (int i : pl->fgroups[g].insts) w += (double)pl->inst[i].npts * pl->inst[i].P * pl->inst[i].nf;
        if (w > most) {
            most = w;
            best = g;
        }
    }
    return best;
}

int build_tables(pr_plan *pl)
{
    const size_t es = esize(pl->dtype);
    const int ninst = pl->ninst;
    const int K = pl->K;
    const VariantInfo *cvi = coarse_info(pl->coarse_v);
    const bool cref = pl->coarse_v == 1;
    for (int i = 0; i < ninst; ++i) {
        const int v = pl->fgroups[pl->inst_group[i]].v;
        if ((v == 1 || fine_info(v)->scratch > 0) && !pl->inst[i].Fscr)
            return fail(PR_EINVAL, "kernel variant changed between workspace query and plan creation");
    }

    pl->slice_base.resize(ninst);
    for (int i = 0, b = 0; i < ninst; ++i) {
        pl->slice_base[i] = b;
        b += pl->inst[i].P;
    }
    auto fine_item = [&](int i, int n) {
        const pr_plan::Inst &in = pl->inst[i];
        ItemDesc it;
        std::memset(&it, 0, sizeof it);
        fill_item(it, pl->probs[i], true);
        it.src0 = slice_ptr(in.Ulo, n, in.npts, es);
        it.dst = slice_ptr(in.Fv, n, in.npts, es);
        it.tmp = slice_ptr(in.Ftmp, n, in.npts, es);
        it.scratch = in.Fscr ? in.Fscr + (size_t)3 * n * in.npts * es : nullptr;
        it.step0 = (int64_t)n * in.nf;
        it.nsteps = in.nf;
        return it;
    };

    // batched fine tables, one per iteration and group (slices n >= k when
    // skipping); items sorted by step count so that the active blocks of
    // step j are a prefix of the grid
    std::vector<ItemDesc> all;
    for (auto &g : pl->fgroups) {
        g.off.assign(std::max(K, 1), 0);
        g.cnt.assign(std::max(K, 1), 0);
        g.active.assign(std::max(K, 1), {});
    }
    // the items of launch group g's slices n in [nlo, nhi) of every instance,
    // laid out and appended to `all`; returns (offset, count, active blocks)
    auto fine_table = [&](const pr_plan::FineGroup &g, int nlo, int nhi, int &off, int &cnt, std::vector<int> &act) {
        std::vector<ItemDesc> items;
        for (int i : g.insts)
            for (int n = nlo; n < std::min(nhi, pl->inst[i].P); ++n) items.push_back(fine_item(i, n));
        std::stable_sort(items.begin(), items.end(),
                         [](const ItemDesc &a, const ItemDesc &b) { return a.nsteps > b.nsteps; });
        layout(items, fine_info(g.v), g.v == 1, 2, 8, g.bpc, pr::fine_occupancy(g.v));
        const int maxsteps = items.empty() ? 0 : items[0].nsteps;
        act.assign(maxsteps, 0);
        for (int j = 0; j < maxsteps; ++j) {
            int blocks = 0;
            for (auto &it : items)
                if (it.nsteps > j) blocks = it.block_begin + it.nblocks;
            act[j] = blocks;
        }
        off = (int)all.size();
        cnt = (int)items.size();
        all.insert(all.end(), items.begin(), items.end());
    };
    for (int k = 0; k < K; ++k)
        for (auto &g : pl->fgroups) fine_table(g, pl->skip ? k : 0, pl->Pmax, g.off[k], g.cnt[k], g.active[k]);
    if (pl->pipe) {
        const int nfg = (int)pl->fgroups.size();
        pl->ptab.assign((size_t)std::max(K, 1) * pl->npg * nfg, {});
        for (int k = 0; k < K; ++k)
            for (int q = 0; q < pl->npg; ++q)
                for (int f = 0; f < nfg; ++f) {
                    pr_plan::PipeTab &t = pl->ptab[((size_t)k * pl->npg + q) * nfg + f];
                    const int nlo = std::max(pl->pg_begin[q], pl->skip ? k : 0);
                    fine_table(pl->fgroups[f], nlo, pl->pg_begin[q + 1], t.off, t.cnt, t.active);
                }
    }
    int rc = upload(pl->fine_tab, all);
    if (rc) return rc;

    // per-slice tables: every (i, n) laid out on its own
    std::vector<ItemDesc> sl;
    pl->slice_index.assign(pl->sumP, 0);
    pl->slice_blocks.clear();
    pl->slice_var.clear();
    for (int i = 0; i < ninst; ++i)
        for (int n = 0; n < pl->inst[i].P; ++n) {
            const int v = pl->fgroups[pl->inst_group[i]].v;
            std::vector<ItemDesc> one{fine_item(i, n)};
            layout(one, fine_info(v), v == 1, 2, 8, 0, pr::fine_occupancy(v));
            pl->slice_index[pl->slice_base[i] + n] = (int)sl.size();
            pl->slice_blocks.push_back(one[0].nblocks);
            pl->slice_var.push_back(v);
            sl.push_back(one[0]);
        }
    rc = upload(pl->slice_tab, sl);
    if (rc) return rc;

    // coarse tables [parity][n]: instances with P_i > n.  With coarsening the
    // sweep runs on the coarsened grid from Cin to Cout, bracketed by the
    // restriction [n] and the interpolation [parity][n] tables.
    const int Pmax = pl->Pmax;
    std::vector<ItemDesc> ct((size_t)2 * Pmax * ninst);
    std::vector<ItemDesc> rt((size_t)Pmax * ninst), pt((size_t)2 * Pmax * ninst);
    pl->coarse_cnt.assign(Pmax, 0);
    pl->coarse_blocks.assign(2 * Pmax, 0);
    pl->coarse_nch.assign(Pmax, 0);
    const int S = coarse_steps_per_launch(pl->coarse_v);
    for (int par = 0; par < 2; ++par)
        for (int n = 0; n < Pmax; ++n) {
            std::vector<ItemDesc> items;
            for (int i = 0; i < ninst; ++i) {
                const pr_plan::Inst &in = pl->inst[i];
                if (n >= in.P) continue;
                ItemDesc it;
                std::memset(&it, 0, sizeof it);
                fill_item(it, coarse_grid(pl->probs[i]), false);
                it.src0 = pl->coarsen ? in.Cin : slice_ptr(in.Ulo, n, in.npts, es);
                it.dst = pl->coarsen ? in.Cout : slice_ptr(in.Gold[par], n, in.npts, es);
                it.tmp = pl->coarsen ? in.Ctmp : in.Gtmp;
                it.step0 = (int64_t)n * in.nc;
                it.nsteps = in.nc;
                items.push_back(it);
                if (pl->coarsen) {
                    const int m = (int)items.size() - 1;
                    ItemDesc x;
                    std::memset(&x, 0, sizeof x);
                    x.nx = pl->probs[i].n[0];
                    x.ny = pl->probs[i].n[1];
                    x.nz = pl->probs[i].n[2];
                    x.src0 = slice_ptr(in.Ulo, n, in.npts, es);
                    x.dst = in.Cin;
                    if (par == 0) rt[(size_t)n * ninst + m] = x;
                    x.src0 = in.Cout;
                    x.dst = slice_ptr(in.Gold[par], n, in.npts, es);
                    pt[((size_t)par * Pmax + n) * ninst + m] = x;
                }
            }
            std::stable_sort(items.begin(), items.end(),
                             [](const ItemDesc &a, const ItemDesc &b) { return a.nsteps > b.nsteps; });
            const int nb = layout(items, cvi, cref, 2, 2 * S, pl->coarse_bpc, pr::coarse_occupancy(pl->coarse_v));
            pl->coarse_blocks[par * Pmax + n] = nb;
            pl->coarse_cnt[n] = (int)items.size();
            pl->coarse_nch[n] = items.empty() ? 0 : (items[0].nsteps + S - 1) / S;
            for (size_t m = 0; m < items.size(); ++m) ct[((size_t)par * Pmax + n) * ninst + m] = items[m];
        }
    rc = upload(pl->coarse_tab, ct);
    if (rc) return rc;
    if (pl->coarsen) {
        rc = upload(pl->rst_tab, rt);
        if (rc) return rc;
        rc = upload(pl->pro_tab, pt);
        if (rc) return rc;
    }

    // pointwise tables
    std::vector<PointItem> assign((size_t)Pmax * ninst), corr((size_t)2 * Pmax * ninst),
        skip((size_t)2 * Pmax * ninst);
    for (int n = 0; n < Pmax; ++n) {
        int m = 0;
        for (int i = 0; i < ninst; ++i) {
            const pr_plan::Inst &in = pl->inst[i];
            if (n >= in.P) continue;
            PointItem a{};
            a.a = slice_ptr(in.Gold[0], n, in.npts, es);
            a.u = in.U + (size_t)(n + 1) * in.npts;
            a.ulo = pl->mixed ? (void *)slice_ptr(in.Ulo, n + 1, in.npts, es) : nullptr;
            a.npts = in.npts;
            assign[(size_t)n * ninst + m] = a;
            for (int par = 0; par < 2; ++par) {
                // iteration k with k % 2 == par: G_new -> Gold[1-par], G_old = Gold[par]
                PointItem c{};
                c.a = slice_ptr(in.Fv, n, in.npts, es);
                c.b = slice_ptr(in.Gold[1 - par], n, in.npts, es);
                c.c = slice_ptr(in.Gold[par], n, in.npts, es);
                c.u = in.U + (size_t)(n + 1) * in.npts;
                c.ulo = pl->mixed ? (void *)slice_ptr(in.Ulo, n + 1, in.npts, es) : nullptr;
                c.partials = in.part + (size_t)n * pr::kNormBlocks * 4;
                c.npts = in.npts;
                corr[((size_t)par * Pmax + n) * ninst + m] = c;
                PointItem s = c;
                s.b = slice_ptr(in.Gold[par], n, in.npts, es);
                skip[((size_t)par * Pmax + n) * ninst + m] = s;
            }
            ++m;
        }
    }
    rc = upload(pl->pt_assign, assign);
    if (rc) return rc;
    rc = upload(pl->pt_corr, corr);
    if (rc) return rc;
    rc = upload(pl->pt_skip, skip);
    if (rc) return rc;

    std::vector<PointItem> fin((size_t)std::max(K, 1) * pl->sumP);
    for (int k = 0; k < K; ++k)
        for (int i = 0; i < ninst; ++i)
            for (int n = 0; n < pl->inst[i].P; ++n) {
                PointItem f{};
                f.partials = pl->inst[i].part + (size_t)n * pr::kNormBlocks * 4;
                f.out4 = pl->dlog + ((size_t)k * pl->sumP + pl->slice_base[i] + n) * 4;
                fin[(size_t)k * pl->sumP + pl->slice_base[i] + n] = f;
            }
    return upload(pl->pt_final, fin);
}

// Start-up coarse run at slice n (after U_n is in place): U_{n+1} = G(U_n).
int enqueue_init_slice(pr_plan *pl, int n, hipStream_t s)
{
    const int ninst = pl->ninst, Pmax = pl->Pmax;
    const int cnt = pl->coarse_cnt[n];
    if (!cnt) return PR_OK;
    const ItemDesc *tab = pl->coarse_tab + (size_t)(0 * Pmax + n) * ninst;
    if (pl->coarsen) HIPCHK(pr::launch_restrict(pl->dtype, pl->rst_tab + (size_t)n * ninst, cnt, s));
    for (int c = 0; c < pl->coarse_nch[n]; ++c)
        HIPCHK(pr::launch_coarse_chunk(pl->coarse_v, pl->dtype, tab, cnt, pl->coarse_blocks[n], c, s));
    if (pl->coarsen)
        HIPCHK(pr::launch_prolong(pl->dtype, pl->iorder, pl->pro_tab + (size_t)(0 * Pmax + n) * ninst, cnt, s));
    HIPCHK(pr::launch_pointwise(pr::kOpAssign, pl->dtype, pl->pt_assign + (size_t)n * ninst, cnt, false, s));
    return PR_OK;
}

// Enqueue the start-up coarse run of Algorithm 1 (after U_0 is in place).
int enqueue_init(pr_plan *pl, hipStream_t s)
{
    for (int n = 0; n < pl->Pmax; ++n) {
        int rc = enqueue_init_slice(pl, n, s);
        if (rc) return rc;
    }
    return PR_OK;
}

int enqueue_fine(pr_plan *pl, int k, hipStream_t s)
{
    if (!pl->per_slice) {
        const int ng = (int)pl->fgroups.size();
        if (ng > 1) {
            HIPCHK(hipEventRecord(pl->fork_ev, s));
            for (int g = 1; g < ng; ++g) HIPCHK(hipStreamWaitEvent(pl->aux[g - 1], pl->fork_ev, 0));
        }
        for (int g = 0; g < ng; ++g) {
            const auto &gr = pl->fgroups[g];
            hipStream_t sg = g == 0 ? s : pl->aux[g - 1];
            const ItemDesc *tab = pl->fine_tab + gr.off[k];
            const std::vector<int> &act = gr.active[k];
            for (int j = 0; j < (int)act.size(); ++j)
                HIPCHK(pr::launch_fine_step(gr.v, pl->dtype, pl->probs[0].fine_order, tab, gr.cnt[k], act[j], j, sg));
        }
        for (int g = 1; g < ng; ++g) {
            HIPCHK(hipEventRecord(pl->join_ev[g - 1], pl->aux[g - 1]));
            HIPCHK(hipStreamWaitEvent(s, pl->join_ev[g - 1], 0));
        }
    } else {
        for (int i = 0; i < pl->ninst; ++i)
            for (int n = (pl->skip ? k : 0); n < pl->inst[i].P; ++n) {
                const int idx = pl->slice_index[pl->slice_base[i] + n];
                const ItemDesc *tab = pl->slice_tab + idx;
                const int nf = pl->inst[i].nf;
                for (int j = 0; j < nf; ++j)
                    HIPCHK(pr::launch_fine_step(pl->slice_var[idx], pl->dtype, pl->probs[i].fine_order, tab, 1,
                                                pl->slice_blocks[idx], j, s));
            }
    }
    return PR_OK;
}

}  // namespace

namespace {

// Iteration k's coarse chain at slice n (Algorithm 1): G of U^{k+1}_n, then
// the correction U^{k+1}_{n+1} = F(U^k_n) + G(U^{k+1}_n) - G(U^k_n).
int enqueue_chain_slice(pr_plan *pl, int k, int n, hipStream_t s)
{
    const int ninst = pl->ninst, Pmax = pl->Pmax;
    const int par = k & 1;
    const int cnt = pl->coarse_cnt[n];
    if (!cnt) return PR_OK;
    if (pl->skip && n == k) {
        // G_n(U^{k+1}_n) would equal G_old bitwise: U^{k+1}_{n+1} = F + 0
        HIPCHK(pr::launch_pointwise(pr::kOpCorrect, pl->dtype, pl->pt_skip + ((size_t)par * Pmax + n) * ninst, cnt,
                                    true, s));
        return PR_OK;
    }
    const int cpar = 1 - par;  // G_new goes to Gold[1 - k%2]
    const ItemDesc *tab = pl->coarse_tab + ((size_t)cpar * Pmax + n) * ninst;
    if (pl->coarsen) HIPCHK(pr::launch_restrict(pl->dtype, pl->rst_tab + (size_t)n * ninst, cnt, s));
    for (int c = 0; c < pl->coarse_nch[n]; ++c)
        HIPCHK(pr::launch_coarse_chunk(pl->coarse_v, pl->dtype, tab, cnt, pl->coarse_blocks[cpar * Pmax + n], c, s));
    if (pl->coarsen)
        HIPCHK(pr::launch_prolong(pl->dtype, pl->iorder, pl->pro_tab + ((size_t)cpar * Pmax + n) * ninst, cnt, s));
    HIPCHK(pr::launch_pointwise(pr::kOpCorrect, pl->dtype, pl->pt_corr + ((size_t)par * Pmax + n) * ninst, cnt, true,
                                s));
    return PR_OK;
}

// The norms that close iteration k: per-slice inter-iterate finals, and d^k
// against the reference.
int enqueue_norms(pr_plan *pl, int k, hipStream_t s, bool with_ref)
{
    HIPCHK(pr::launch_defect_final(pl->pt_final + (size_t)k * pl->sumP, pl->sumP, s));
    if (with_ref) {
        HIPCHK(pr::launch_defect_partials(PR_FP64, PR_FP64, pl->io_ref + (size_t)k * pl->ninst, pl->ninst, s));
        HIPCHK(pr::launch_defect_final(pl->io_ref + (size_t)k * pl->ninst, pl->ninst, s));
    }
    return PR_OK;
}

int enqueue_iteration(pr_plan *pl, int k, hipStream_t s, bool with_ref)
{
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[2 + 3 * k], s));
    int rc = enqueue_fine(pl, k, s);
    if (rc) return rc;
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[3 + 3 * k], s));
    for (int n = pl->skip ? k : 0; n < pl->Pmax; ++n) {
        rc = enqueue_chain_slice(pl, k, n, s);
        if (rc) return rc;
    }
    rc = enqueue_norms(pl, k, s, with_ref);
    if (rc) return rc;
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[4 + 3 * k], s));
    return PR_OK;
}

int enqueue_head(pr_plan *pl, hipStream_t s)
{
    HIPCHK(pr::launch_pointwise(pr::kOpCopy64, pl->dtype, pl->io_u0, pl->ninst, false, s));
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[0], s));
    int rc = enqueue_init(pl, s);
    if (rc) return rc;
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[1], s));
    return PR_OK;
}

int enqueue_tail(pr_plan *pl, hipStream_t s)
{
    HIPCHK(pr::launch_pointwise(pr::kOpCopy64, pl->dtype, pl->io_uT, pl->ninst, false, s));
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev.back(), s));
    return PR_OK;
}

// F of iteration k on slice group q: for every launch group with slices in
// q, on that group's F stream, after the chain has made the group ready.
int enqueue_pipe_fine(pr_plan *pl, int k, int q)
{
    const int nfg = (int)pl->fgroups.size();
    const size_t e = (size_t)k * pl->npg + q;
    for (int f = 0; f < nfg; ++f) {
        const size_t t = e * nfg + f;
        const pr_plan::PipeTab &tb = pl->ptab[t];
        if (!tb.cnt) continue;
        const auto &gr = pl->fgroups[f];
        hipStream_t fs = pl->fstream[f];
        HIPCHK(hipStreamWaitEvent(fs, pl->ready[e], 0));
        if (pl->timed) HIPCHK(hipEventRecord(pl->tbeg[t], fs));
        for (int j = 0; j < (int)tb.active.size(); ++j) {
            HIPCHK(pr::launch_fine_step(gr.v, pl->dtype, pl->probs[0].fine_order, pl->fine_tab + tb.off, tb.cnt,
                                        tb.active[j], j, fs));
            if (j == 0) HIPCHK(hipEventRecord(pl->first[t], fs));
        }
        if (pl->timed) HIPCHK(hipEventRecord(pl->tend[t], fs));
        HIPCHK(hipEventRecord(pl->done[t], fs));
    }
    return PR_OK;
}

// The solve's stream waits until F of (k, q) has run all its steps (which =
// done) or its first step (which = first), for every launch group in q.
int wait_pipe_fine(pr_plan *pl, int k, int q, bool first, hipStream_t s)
{
    const int nfg = (int)pl->fgroups.size();
    for (int f = 0; f < nfg; ++f) {
        const size_t t = ((size_t)k * pl->npg + q) * nfg + f;
        if (pl->ptab[t].cnt) HIPCHK(hipStreamWaitEvent(s, first ? pl->first[t] : pl->done[t], 0));
    }
    return PR_OK;
}

// The pipelined schedule (Section 2.2.1, Algorithm 1 with each slice's F
// started as soon as its input is final).  Dependencies, per slice group q:
//   F(k, q) after the chain of iteration k-1 has left q (U^k_n of q final, and
//     F^{k-1}_n of q consumed by its corrections; for k = 0, after the
//     start-up run has set U^0_n of q);
//   the chain of iteration k enters q after F(k, q) is done;
//   its correction at the last slice of q, which writes U^{k+1} of the first
//     slice of q+1, waits until F(k, q+1) has run its first step (the only
//     step that reads U^k there).
// Every buffer is then read and written in the order of the phase-by-phase
// schedule, so the results are bitwise the same.
int enqueue_pipelined(pr_plan *pl, hipStream_t s, bool with_ref)
{
    const int npg = pl->npg, K = pl->K, Pmax = pl->Pmax;
    const std::vector<int> &b = pl->pg_begin;
    int rc;
    HIPCHK(pr::launch_pointwise(pr::kOpCopy64, pl->dtype, pl->io_u0, pl->ninst, false, s));
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[0], s));
    // start-up run: group q is ready once U^0 of its last slice is set, i.e.
    // after slice b[q+1]-2 (U_0 is set before the run)
    int q = 0;
    for (int n = -1; n < Pmax; ++n) {
        if (n >= 0) {
            rc = enqueue_init_slice(pl, n, s);
            if (rc) return rc;
        }
        for (; q < npg && b[q + 1] - 2 <= n; ++q)
            if (K > 0) HIPCHK(hipEventRecord(pl->ready[q], s));
    }
    if (pl->timed) HIPCHK(hipEventRecord(pl->ev[1], s));
    if (K > 0) {
        rc = enqueue_pipe_fine(pl, 0, 0);
        if (rc) return rc;
    }
    for (int k = 0; k < K; ++k) {
        const int nstart = pl->skip ? k : 0;
        for (q = 0; q < npg; ++q) {
            if (q + 1 < npg) {
                rc = enqueue_pipe_fine(pl, k, q + 1);
                if (rc) return rc;
            }
            if (pl->timed && q == 0) HIPCHK(hipEventRecord(pl->ev[2 + 3 * k], s));
            rc = wait_pipe_fine(pl, k, q, false, s);
            if (rc) return rc;
            if (pl->timed && q == 0) HIPCHK(hipEventRecord(pl->ev[3 + 3 * k], s));
            for (int n = std::max(b[q], nstart); n < b[q + 1]; ++n) {
                if (n == b[q + 1] - 1 && q + 1 < npg) {
                    rc = wait_pipe_fine(pl, k, q + 1, true, s);
                    if (rc) return rc;
                }
                rc = enqueue_chain_slice(pl, k, n, s);
                if (rc) return rc;
            }
            if (k + 1 < K) HIPCHK(hipEventRecord(pl->ready[(size_t)(k + 1) * npg + q], s));
        }
        rc = enqueue_norms(pl, k, s, with_ref);
        if (rc) return rc;
        if (pl->timed) HIPCHK(hipEventRecord(pl->ev[4 + 3 * k], s));
        if (k + 1 < K) {
            rc = enqueue_pipe_fine(pl, k + 1, 0);
            if (rc) return rc;
        }
    }
    return enqueue_tail(pl, s);
}

int enqueue_all(pr_plan *pl, hipStream_t s, bool with_ref)
{
    if (pl->pipe) return enqueue_pipelined(pl, s, with_ref);
    int rc = enqueue_head(pl, s);
    if (rc) return rc;
    for (int k = 0; k < pl->K; ++k) {
        rc = enqueue_iteration(pl, k, s, with_ref);
        if (rc) return rc;
    }
    return enqueue_tail(pl, s);
}

int count_launches(const pr_plan *pl, double *nf, double *ng)
{
    double f = 0, g = 0;
    for (int k = 0; k < pl->iters_done; ++k) {
        if (pl->pipe) {
            const size_t per_k = (size_t)pl->npg * pl->fgroups.size();
            for (size_t t = 0; t < per_k; ++t) f += (double)pl->ptab[(size_t)k * per_k + t].active.size();
        } else if (!pl->per_slice) {
            for (const auto &gr : pl->fgroups) f += (double)gr.active[k].size();
        } else {
            for (int i = 0; i < pl->ninst; ++i)
                for (int n = (pl->skip ? k : 0); n < pl->inst[i].P; ++n) f += pl->inst[i].nf;
        }
        for (int n = (pl->skip ? k + 1 : 0); n < pl->Pmax; ++n) g += pl->coarse_nch[n];
    }
    for (int n = 0; n < pl->Pmax; ++n) g += pl->coarse_nch[n];
    *nf = f;
    *ng = g;
    return PR_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char *pr_last_error(void) { return g_err.c_str(); }

const char *pr_version(void) { return "pr 0.1 gfx950"; }

int pr_check_stability(const pr_problem *prob, double *fine_margin, double *coarse_margin)
{
    int rc = validate_problem(prob, false);
    if (rc) return rc;
    double fm = 0, cm = 0;
    margins_cached(*prob, &fm, &cm);
    if (fine_margin) *fine_margin = fm;
    if (coarse_margin) *coarse_margin = cm;
    if (fm > 1.0 + 1e-12 || cm > 1.0 + 1e-12)
        return fail(PR_EUNSTABLE, "unstable: fine margin %.6g, coarse margin %.6g", fm, cm);
    return PR_OK;
}

size_t pr_sweep_workspace_bytes(const pr_problem *prob, int32_t dtype, int32_t batch)
{
    if (validate_problem(prob, false) || batch < 1 || (dtype != PR_FP32 && dtype != PR_FP64)) return 0;
    return sweep_ws(*prob, dtype, batch, g_fine_forced == 1);
}

int pr_fine_sweep(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_in, void *u_out,
                  const int64_t *step0, int32_t nsteps, void *ws, size_t ws_bytes, void *stream)
{
    return sweep_common(prob, dtype, batch, u_in, u_out, step0, nsteps, ws, ws_bytes, stream, true);
}

int pr_coarse_sweep(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_in, void *u_out,
                    const int64_t *step0, int32_t nsteps, void *ws, size_t ws_bytes, void *stream)
{
    return sweep_common(prob, dtype, batch, u_in, u_out, step0, nsteps, ws, ws_bytes, stream, false);
}

size_t pr_transfer_workspace_bytes(int32_t batch)
{
    if (batch < 1) return 0;
    return align256((size_t)batch * sizeof(ItemDesc));
}

static int transfer_common(const pr_problem *prob, int dtype, int order, int batch, const void *in, void *out,
                           void *ws, size_t ws_bytes, void *stream, bool prolong)
{
    if (!prob) return fail(PR_EINVAL, "problem is NULL");
    pr_problem p = *prob;
    p.flags = PR_COARSEN_G;   // only the grid matters here
    int rc = validate_problem(&p, false);
    if (rc) return rc;
    if (dtype != PR_FP32 && dtype != PR_FP64) return fail(PR_EINVAL, "dtype must be PR_FP32 or PR_FP64");
    if (prolong && order != 1 && order != 3) return fail(PR_EINVAL, "interpolation order must be 1 or 3");
    if (batch < 1) return fail(PR_EINVAL, "batch must be >= 1");
    if (!in || !out) return fail(PR_EINVAL, "NULL field pointer");
    const size_t fb = (size_t)npts_of(p) * esize(dtype), cb = fb / 8;
    const size_t inb = (prolong ? cb : fb) * batch, outb = (prolong ? fb : cb) * batch;
    const char *a = (const char *)in, *o = (const char *)out;
    if (a < o + outb && o < a + inb) return fail(PR_EINVAL, "input and output overlap");
    const size_t need = pr_transfer_workspace_bytes(batch);
    if (!ws || ws_bytes < need) return fail(PR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    rc = device_ready();
    if (rc) return rc;
    std::vector<ItemDesc> items(batch);
    for (int b = 0; b < batch; ++b) {
        ItemDesc &it = items[b];
        std::memset(&it, 0, sizeof it);
        it.nx = p.n[0];
        it.ny = p.n[1];
        it.nz = p.n[2];
        it.src0 = a + b * (prolong ? cb : fb);
        it.dst = (char *)out + b * (prolong ? fb : cb);
    }
    hipStream_t s = (hipStream_t)stream;
    ItemDesc *table = (ItemDesc *)ws;
    HIPCHK(pr::launch_write_items(items.data(), batch, table, s));
    if (prolong) HIPCHK(pr::launch_prolong(dtype, order, table, batch, s));
    else HIPCHK(pr::launch_restrict(dtype, table, batch, s));
    return PR_OK;
}

int pr_restrict(const pr_problem *prob, int32_t dtype, int32_t batch, const void *u_fine, void *u_coarse, void *ws,
                size_t ws_bytes, void *stream)
{
    return transfer_common(prob, dtype, 1, batch, u_fine, u_coarse, ws, ws_bytes, stream, false);
}

int pr_prolong(const pr_problem *prob, int32_t dtype, int32_t order, int32_t batch, const void *u_coarse,
               void *u_fine, void *ws, size_t ws_bytes, void *stream)
{
    return transfer_common(prob, dtype, order, batch, u_coarse, u_fine, ws, ws_bytes, stream, true);
}

int pr_parareal_update(int64_t npts, int32_t batch, int32_t sweep_dtype, const void *f_new, const void *g_new,
                       const void *g_old, double *u_out, void *u_out_lo, void *stream)
{
    if (npts < 0 || batch < 1) return fail(PR_EINVAL, "npts must be >= 0 and batch >= 1");
    if (sweep_dtype != PR_FP32 && sweep_dtype != PR_FP64) return fail(PR_EINVAL, "bad sweep dtype");
    if (!f_new || !g_new || !g_old || !u_out) return fail(PR_EINVAL, "NULL field pointer");
    if (npts == 0) return PR_OK;
    int rc = device_ready();
    if (rc) return rc;
    PointItem it{};
    it.a = f_new;
    it.b = g_new;
    it.c = g_old;
    it.u = u_out;
    it.ulo = u_out_lo;
    it.npts = npts * batch;
    HIPCHK(pr::launch_pointwise_inline(pr::kOpCorrect, sweep_dtype, it, (hipStream_t)stream));
    return PR_OK;
}

size_t pr_defect_workspace_bytes(int32_t batch)
{
    if (batch < 1) return 0;
    return align256((size_t)batch * sizeof(PointItem)) + (size_t)batch * pr::kNormBlocks * 4 * sizeof(double);
}

}  // extern "C"

namespace {

int defect_args(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                const double *out4)
{
    if (npts < 1 || batch < 1) return fail(PR_EINVAL, "npts and batch must be >= 1");
    if ((xd != PR_FP32 && xd != PR_FP64) || (rd != PR_FP32 && rd != PR_FP64)) return fail(PR_EINVAL, "bad dtype");
    if (!x || !ref || !out4) return fail(PR_EINVAL, "NULL pointer");
    return PR_OK;
}

// The norms of `batch` field pairs with the item table at `table` and the
// block partials at `part` (kNormBlocks * 4 doubles per pair).  Every partial
// is written by the first pass before the second reads it, so nothing needs
// clearing.
// `items` is host storage for `batch` descriptors.
int defect_enqueue(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                   double *out4, PointItem *items, PointItem *table, double *part, hipStream_t s)
{
    for (int b = 0; b < batch; ++b) {
        PointItem &it = items[b];
        it = PointItem{};
        it.a = (const char *)x + (size_t)b * npts * esize(xd);
        it.b = (const char *)ref + (size_t)b * npts * esize(rd);
        it.partials = part + (size_t)b * pr::kNormBlocks * 4;
        it.out4 = out4 + 4 * (size_t)b;
        it.npts = npts;
    }
    HIPCHK(pr::launch_write_points(items, batch, table, s));
    HIPCHK(pr::launch_defect_partials(xd, rd, table, batch, s));
    HIPCHK(pr::launch_defect_final(table, batch, s));
    return PR_OK;
}

}  // namespace

extern "C" {

int pr_defect_norm(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                   double *out4, void *ws, size_t ws_bytes, void *stream)
{
    int rc = defect_args(npts, batch, xd, x, rd, ref, out4);
    if (rc) return rc;
    const size_t need = pr_defect_workspace_bytes(batch);
    if (!ws || ws_bytes < need) return fail(PR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    rc = device_ready();
    if (rc) return rc;
    char *w = (char *)ws;
    PointItem *table = (PointItem *)w;
    double *part = (double *)(w + align256((size_t)batch * sizeof(PointItem)));
    std::vector<PointItem> items(batch);
    return defect_enqueue(npts, batch, xd, x, rd, ref, out4, items.data(), table, part, (hipStream_t)stream);
}

}  // extern "C"

// ---- pr_defect_norm_static: the norms without a caller workspace ----------
//
// The item table and the block partials live in a file-scope device array
// (one copy per GPU, held until the process ends).  In host code `scratch`
// names a host-side stand-in, not device memory: the device address of each
// GPU's copy is taken once per device with hipGetSymbolAddress and only that
// address reaches the kernels.
namespace {

constexpr size_t kStaticTableBytes = ((size_t)PR_DEFECT_STATIC_MAX_BATCH * sizeof(PointItem) + 255) & ~(size_t)255;
constexpr size_t kStaticScratchBytes =
    kStaticTableBytes + (size_t)PR_DEFECT_STATIC_MAX_BATCH * pr::kNormBlocks * 4 * sizeof(double);

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call on that device, with the device current).
int static_scratch(void **out)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PR_EDEVICE, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PR_EDEVICE, "hipGetSymbolAddress returned NULL for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PR_OK;
}

}  // namespace

extern "C" {

size_t pr_defect_static_scratch_bytes(void) { return kStaticScratchBytes; }

int pr_copy_probe(const void *src, void *dst, size_t bytes, int32_t variant, int32_t blocks_per_cu, void *stream)
{
    if (!src || !dst) return fail(PR_EINVAL, "NULL pointer");
    if (bytes == 0 || bytes % 16) return fail(PR_EINVAL, "bytes must be a positive multiple of 16");
    if (((uintptr_t)src | (uintptr_t)dst) % 16) return fail(PR_EINVAL, "buffers must be 16-byte aligned");
    const char *a = (const char *)src, *o = (const char *)dst;
    if (a < o + bytes && o < a + bytes) return fail(PR_EINVAL, "source and destination overlap");
    if (variant < 0 || variant > 3) return fail(PR_EINVAL, "variant must be 0..3");
    if (blocks_per_cu < 0 || blocks_per_cu > 64) return fail(PR_EINVAL, "blocks_per_cu must be 0..64");
    int rc = device_ready();
    if (rc) return rc;
    const int blocks = g_num_cus * (blocks_per_cu ? blocks_per_cu : 8);
    HIPCHK(pr::launch_copy_probe(variant, src, dst, bytes, blocks, (hipStream_t)stream));
    return PR_OK;
}

int pr_defect_norm_static(int64_t npts, int32_t batch, int32_t xd, const void *x, int32_t rd, const void *ref,
                          double *out4, void *stream)
{
    int rc = defect_args(npts, batch, xd, x, rd, ref, out4);
    if (rc) return rc;
    if (batch > PR_DEFECT_STATIC_MAX_BATCH)
        return fail(PR_EINVAL, "batch %d exceeds the %d field pairs the static scratch holds; use pr_defect_norm",
                    batch, PR_DEFECT_STATIC_MAX_BATCH);
    rc = device_ready();
    if (rc) return rc;
    void *base = nullptr;
    rc = static_scratch(&base);
    if (rc) return rc;
    char *w = (char *)base;
    PointItem *table = (PointItem *)w;
    double *part = (double *)(w + kStaticTableBytes);
    PointItem items[PR_DEFECT_STATIC_MAX_BATCH];   // host staging of the descriptors, no heap
    return defect_enqueue(npts, batch, xd, x, rd, ref, out4, items, table, part, (hipStream_t)stream);
}

size_t pr_plan_workspace_bytes(const pr_problem *probs, int32_t ninst, int32_t mode)
{
    if (validate_plan_args(probs, ninst, mode)) return 0;
    return plan_layout(probs, ninst, mode, nullptr, nullptr);
}

int pr_plan_create(const pr_problem *probs, int32_t ninst, int32_t mode, void *ws, size_t ws_bytes, pr_plan **out)
{
    if (!out) return fail(PR_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_plan_args(probs, ninst, mode);
    if (rc) return rc;
    const size_t need = plan_layout(probs, ninst, mode, nullptr, nullptr);
    if (!ws || ws_bytes < need) return fail(PR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    rc = device_ready();
    if (rc) return rc;

    pr_plan *pl = new pr_plan();
    pl->ninst = ninst;
    pl->mode = mode;
    pl->mixed = (mode & PR_MODE_MIXED) != 0;
    pl->per_slice = (mode & PR_MODE_PER_SLICE) != 0;
    pl->dtype = pl->mixed ? PR_FP32 : PR_FP64;
    pl->K = probs[0].K;
    pl->flags = probs[0].flags;
    pl->skip = (pl->flags & PR_SKIP_CONVERGED) != 0;
    pl->early = (pl->flags & PR_EARLY_STOP) != 0;
    pl->timed = (mode & PR_MODE_TIMED) != 0;
    pl->graph = (mode & PR_MODE_GRAPH) != 0 && !pl->early && !pl->timed;
    pl->probs.assign(probs, probs + ninst);
    pl->coarsen = (pl->flags & PR_COARSEN_G) != 0;
    pl->iorder = interp_order(probs[0]);

    for (int i = 0; i < ninst; ++i)
        if (probs[i].fine_order != probs[0].fine_order) {
            delete pl;
            return fail(PR_EUNSUPPORTED, "instances of one plan must share fine_order");
        }
    // F: every instance takes the choice for its own grid, at the batch of
    // all slices of the instances with that grid; instances with the same
    // choice share one launch per step (a group).  A forced variant must
    // apply to every instance and gives a single group.
    pl->inst_group.assign(ninst, 0);
    for (int i = 0; i < ninst; ++i) {
        Choice c;
        if (g_fine_forced) {
            c = Choice{g_fine_forced, g_bpc_forced};
            if (!fine_applicable(c.v, pl->dtype, probs[i].fine_order, probs[i])) {
                delete pl;
                return fail(PR_EUNSUPPORTED, "forced kernel variant does not apply to every instance");
            }
        } else {
            int batch = 0;
            for (int j = 0; j < ninst; ++j)
                if (probs[j].n[0] == probs[i].n[0] && probs[j].n[1] == probs[i].n[1] && probs[j].n[2] == probs[i].n[2])
                    batch += probs[j].P;
            c = pick_fine(probs[i], pl->dtype, batch);
            if (c.v < 1 || !fine_applicable(c.v, pl->dtype, probs[i].fine_order, probs[i]))
                c = Choice{pick_fine_default(probs[i], pl->dtype, batch), 0};
            if (c.v < 1) {
                delete pl;
                return fail(PR_EUNSUPPORTED, "instance %d: no fine kernel variant for this grid", i);
            }
        }
        int g = 0;
        while (g < (int)pl->fgroups.size() && !(pl->fgroups[g].v == c.v && pl->fgroups[g].bpc == c.bpc)) ++g;
        if (g == (int)pl->fgroups.size()) {
            pl->fgroups.emplace_back();
            pl->fgroups.back().v = c.v;
            pl->fgroups.back().bpc = c.bpc;
        }
        pl->fgroups[g].insts.push_back(i);
        pl->inst_group[i] = g;
    }
    // G: one fused variant for all instances (the chain's launches are per
    // slice boundary): the choice for instance 0 if it applies to every
    // instance, else the built-in choice for instances of different widths
    const Choice cch = pick_coarse(coarse_grid(probs[0]), pl->dtype, ninst);
    int cv = cch.v;
    bool cok = cv >= 1;
    bool all_even_c = true;
    for (int i = 0; i < ninst; ++i) {
        cok = cok && coarse_applicable(cv, pl->dtype, coarse_grid(probs[i]));
        all_even_c = all_even_c && coarse_grid(probs[i]).n[0] % 2 == 0;
    }
    if (!cok) cv = g_coarse_forced ? -1 : pick_coarse_mixed(pl->dtype, all_even_c);
    if (cv < 1) {
        delete pl;
        return fail(PR_EUNSUPPORTED, "forced kernel variant does not apply to every instance");
    }
    pl->coarse_v = cv;
    pl->coarse_bpc = cok ? cch.bpc : 0;

    plan_layout(probs, ninst, mode, (char *)ws, pl);
    pl->pipe = (mode & PR_MODE_PIPELINED) != 0;
    if (pl->pipe) {
        const int want = (mode >> 16) & 255;
        pl->npg = std::min(std::max(want > 0 ? want : 2, 1), pl->Pmax);
        pl->pg_begin.resize(pl->npg + 1);
        for (int q = 0; q <= pl->npg; ++q) pl->pg_begin[q] = (int)((int64_t)q * pl->Pmax / pl->npg);
    }
    rc = build_tables(pl);
    if (rc) {
        delete pl;
        return rc;
    }
    if (pl->fgroups.size() > 1 && !pl->per_slice) {
        hipError_t er = hipEventCreateWithFlags(&pl->fork_ev, hipEventDisableTiming);
        for (size_t g = 1; g < pl->fgroups.size() && er == hipSuccess; ++g) {
            hipStream_t st = nullptr;
            hipEvent_t e = nullptr;
            er = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (er == hipSuccess) pl->aux.push_back(st);
            if (er == hipSuccess) er = hipEventCreateWithFlags(&e, hipEventDisableTiming);
            if (er == hipSuccess) pl->join_ev.push_back(e);
        }
        if (er != hipSuccess) {
            pr_plan_destroy(pl);
            return fail(PR_EDEVICE, "stream or event creation failed: %s", hipGetErrorString(er));
        }
    }
    if (pl->pipe) {
        const size_t nt = pl->ptab.size();
        hipError_t er = hipSuccess;
        for (size_t f = 0; f < pl->fgroups.size() && er == hipSuccess; ++f) {
            hipStream_t st = nullptr;
            er = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (er == hipSuccess) pl->fstream.push_back(st);
        }
        auto make = [&](std::vector<hipEvent_t> &v, size_t n, bool timing) {
            for (size_t i = 0; i < n && er == hipSuccess; ++i) {
                hipEvent_t e = nullptr;
                er = timing ? hipEventCreate(&e) : hipEventCreateWithFlags(&e, hipEventDisableTiming);
                if (er == hipSuccess) v.push_back(e);
            }
        };
        make(pl->ready, (size_t)std::max(pl->K, 1) * pl->npg, false);
        make(pl->first, nt, false);
        make(pl->done, nt, false);
        if (pl->timed) {
            make(pl->tbeg, nt, true);
            make(pl->tend, nt, true);
        }
        if (er != hipSuccess) {
            pr_plan_destroy(pl);
            return fail(PR_EDEVICE, "stream or event creation failed: %s", hipGetErrorString(er));
        }
    }
    if (pl->timed) {
        pl->ev.resize(3 + 3 * std::max(pl->K, 1));
        for (auto &e : pl->ev) {
            hipError_t er = hipEventCreate(&e);
            if (er != hipSuccess) {
                pr_plan_destroy(pl);
                return fail(PR_EDEVICE, "hipEventCreate failed: %s", hipGetErrorString(er));
            }
        }
    }
    *out = pl;
    return PR_OK;
}

void pr_plan_destroy(pr_plan *plan)
{
    if (!plan) return;
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph_h) (void)hipGraphDestroy(plan->graph_h);
    for (auto &e : plan->ev)
        if (e) (void)hipEventDestroy(e);
    if (plan->own) (void)hipStreamDestroy(plan->own);
    for (auto st : plan->aux) (void)hipStreamDestroy(st);
    for (auto e : plan->join_ev) (void)hipEventDestroy(e);
    if (plan->fork_ev) (void)hipEventDestroy(plan->fork_ev);
    for (auto st : plan->fstream) (void)hipStreamDestroy(st);
    for (auto *v : {&plan->ready, &plan->first, &plan->done, &plan->tbeg, &plan->tend})
        for (auto e : *v) (void)hipEventDestroy(e);
    delete plan;
}

int pr_plan_iterations(const pr_plan *plan) { return plan ? plan->iters_done : 0; }

int pr_plan_kernel_variants(const pr_plan *plan, int32_t *fine_variant, int32_t *coarse_variant)
{
    if (!plan) return fail(PR_EINVAL, "plan is NULL");
    if (fine_variant) *fine_variant = plan->fgroups[primary_group(plan)].v;
    if (coarse_variant) *coarse_variant = plan->coarse_v;
    return PR_OK;
}

int pr_plan_fine_groups(const pr_plan *plan, int32_t max, int32_t *count, int32_t *variant,
                        int32_t *blocks_per_cu, int32_t *instances)
{
    if (!plan || !count) return fail(PR_EINVAL, "NULL argument");
    if (max < 0) return fail(PR_EINVAL, "max must be >= 0");
    if (max > 0 && (!variant || !blocks_per_cu || !instances)) return fail(PR_EINVAL, "NULL output array");
    const int ng = (int)plan->fgroups.size();
    *count = ng;
    for (int g = 0; g < ng && g < max; ++g) {
        variant[g] = plan->fgroups[g].v;
        blocks_per_cu[g] = plan->fgroups[g].bpc;
        instances[g] = (int32_t)plan->fgroups[g].insts.size();
    }
    return PR_OK;
}

int pr_plan_slice_state(const pr_plan *plan, int32_t inst, int32_t n, const double **out)
{
    if (!plan || !out) return fail(PR_EINVAL, "NULL argument");
    if (inst < 0 || inst >= plan->ninst) return fail(PR_EINVAL, "instance out of range");
    if (n < 0 || n > plan->inst[inst].P) return fail(PR_EINVAL, "slice boundary out of range");
    *out = plan->inst[inst].U + (size_t)n * plan->inst[inst].npts;
    return PR_OK;
}

int pr_plan_timings(const pr_plan *plan, double *out6)
{
    if (!plan || !out6) return fail(PR_EINVAL, "NULL argument");
    if (!plan->timed) return fail(PR_EINVAL, "plan was not created with PR_MODE_TIMED");
    for (int i = 0; i < 6; ++i) out6[i] = plan->timings[i];
    return PR_OK;
}

int pr_parareal_solve(pr_plan *pl, const double *const *u0, double *const *uT, const double *const *ref, double *log,
                      void *stream)
{
    if (!pl) return fail(PR_EINVAL, "plan is NULL");
    if (!u0 || !uT) return fail(PR_EINVAL, "u0/uT is NULL");
    for (int i = 0; i < pl->ninst; ++i) {
        if (!u0[i] || !uT[i]) return fail(PR_EINVAL, "u0[%d]/uT[%d] is NULL", i, i);
        if (ref && !ref[i]) return fail(PR_EINVAL, "ref[%d] is NULL", i);
    }
    int rc = device_ready();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int ninst = pl->ninst, K = pl->K;
    const bool with_ref = ref != nullptr;

    // per-solve I/O tables
    std::vector<PointItem> io(ninst), ioT(ninst);
    for (int i = 0; i < ninst; ++i) {
        const pr_plan::Inst &in = pl->inst[i];
        io[i] = PointItem{};
        io[i].a = u0[i];
        io[i].u = in.U;
        io[i].ulo = pl->mixed ? (void *)in.Ulo : nullptr;
        io[i].npts = in.npts;
        ioT[i] = PointItem{};
        ioT[i].a = in.U + (size_t)in.P * in.npts;
        ioT[i].u = uT[i];
        ioT[i].npts = in.npts;
    }
    HIPCHK(pr::launch_write_points(io.data(), ninst, pl->io_u0, s));
    HIPCHK(pr::launch_write_points(ioT.data(), ninst, pl->io_uT, s));
    if (with_ref && K > 0) {
        std::vector<PointItem> ir((size_t)K * ninst);
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < ninst; ++i) {
                const pr_plan::Inst &in = pl->inst[i];
                PointItem r{};
                r.a = in.U + (size_t)in.P * in.npts;
                r.b = ref[i];
                r.partials = in.refpart;
                r.out4 = pl->dlog_ref + ((size_t)k * ninst + i) * 4;
                r.npts = in.npts;
                ir[(size_t)k * ninst + i] = r;
            }
        HIPCHK(pr::launch_write_points(ir.data(), (int)ir.size(), pl->io_ref, s));
    }

    pl->iters_done = K;
    if (pl->graph) {
        if (!pl->exec || pl->had_ref_graph != with_ref) {
            if (pl->exec) {
                HIPCHK(hipGraphExecDestroy(pl->exec));
                pl->exec = nullptr;
            }
            if (pl->graph_h) {
                HIPCHK(hipGraphDestroy(pl->graph_h));
                pl->graph_h = nullptr;
            }
            if (!pl->own) HIPCHK(hipStreamCreateWithFlags(&pl->own, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(pl->own, hipStreamCaptureModeThreadLocal));
            rc = enqueue_all(pl, pl->own, with_ref);
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(pl->own, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ee != hipSuccess) return fail(PR_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ee));
            pl->graph_h = g;
            HIPCHK(hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0));
            pl->had_ref_graph = with_ref;
        }
        HIPCHK(hipGraphLaunch(pl->exec, s));
    } else if (pl->early) {
        rc = enqueue_head(pl, s);
        if (rc) return rc;
        pl->iters_done = 0;
        for (int k = 0; k < K; ++k) {
            rc = enqueue_iteration(pl, k, s, with_ref);
            if (rc) return rc;
            pl->iters_done = k + 1;
            HIPCHK(hipStreamSynchronize(s));
            bool all = true;
            for (int i = 0; i < ninst; ++i) {
                double e4[4];
                const int slot = pl->slice_base[i] + pl->inst[i].P - 1;
                HIPCHK(hipMemcpy(e4, pl->dlog + ((size_t)k * pl->sumP + slot) * 4, sizeof e4, hipMemcpyDeviceToHost));
                if (!(e4[0] <= pl->probs[0].tol * e4[1])) all = false;
            }
            if (all) break;
        }
        rc = enqueue_tail(pl, s);
        if (rc) return rc;
    } else {
        rc = enqueue_all(pl, s, with_ref);
        if (rc) return rc;
    }
    HIPCHK(hipStreamSynchronize(s));

    // logs
    const int Kd = pl->iters_done;
    std::vector<double> dl((size_t)std::max(K, 1) * pl->sumP * 4, 0.0), dr((size_t)std::max(K, 1) * ninst * 4, 0.0);
    if (Kd > 0) {
        HIPCHK(hipMemcpy(dl.data(), pl->dlog, (size_t)Kd * pl->sumP * 4 * sizeof(double), hipMemcpyDeviceToHost));
        if (with_ref)
            HIPCHK(hipMemcpy(dr.data(), pl->dlog_ref, (size_t)Kd * ninst * 4 * sizeof(double), hipMemcpyDeviceToHost));
    }
    bool finite = true;
    for (int i = 0; i < ninst; ++i) {
        const int P = pl->inst[i].P;
        for (int k = 0; k < Kd; ++k) {
            double row[12] = {0};
            const double *fin = &dl[((size_t)k * pl->sumP + pl->slice_base[i] + P - 1) * 4];
            for (int c = 0; c < 4; ++c) row[c] = fin[c];
            for (int n = 0; n < P; ++n) {
                const bool computed = !pl->skip || n >= k;
                const int kk = computed ? k : n;  // slice n last changed in iteration n
                const double *e = &dl[((size_t)kk * pl->sumP + pl->slice_base[i] + n) * 4];
                const double dmax = computed ? e[0] : 0.0, dsum = computed ? e[2] : 0.0;
                row[4] = nan_max(row[4], dmax);
                row[5] = nan_max(row[5], e[1]);
                row[6] += dsum;
                row[7] += e[3];
            }
            if (with_ref)
                for (int c = 0; c < 4; ++c) row[8 + c] = dr[((size_t)k * ninst + i) * 4 + c];
            for (int c = 0; c < 12; ++c)
                if (!std::isfinite(row[c])) finite = false;
            if (log)
                for (int c = 0; c < 12; ++c) log[((size_t)i * K + k) * 12 + c] = row[c];
        }
    }
    if (pl->timed) {
        float ms = 0;
        double f = 0, g = 0;
        HIPCHK(hipEventElapsedTime(&ms, pl->ev[0], pl->ev[1]));
        pl->timings[2] = ms;
        const int nfg = (int)pl->fgroups.size();
        for (int k = 0; k < Kd; ++k) {
            if (pl->pipe) {
                // span of each slice group's F over its launch groups' streams
                for (int q = 0; q < pl->npg; ++q) {
                    double lo = 1e300, hi = -1e300;
                    for (int ff = 0; ff < nfg; ++ff) {
                        const size_t t = ((size_t)k * pl->npg + q) * nfg + ff;
                        if (!pl->ptab[t].cnt) continue;
                        HIPCHK(hipEventElapsedTime(&ms, pl->ev[0], pl->tbeg[t]));
                        lo = std::min(lo, (double)ms);
                        HIPCHK(hipEventElapsedTime(&ms, pl->ev[0], pl->tend[t]));
                        hi = std::max(hi, (double)ms);
                    }
                    if (hi > lo) f += hi - lo;
                }
            } else {
                HIPCHK(hipEventElapsedTime(&ms, pl->ev[2 + 3 * k], pl->ev[3 + 3 * k]));
                f += ms;
            }
            HIPCHK(hipEventElapsedTime(&ms, pl->ev[3 + 3 * k], pl->ev[4 + 3 * k]));
            g += ms;
        }
        pl->timings[0] = f;
        pl->timings[1] = g;
        double nf = 0, ng = 0;
        count_launches(pl, &nf, &ng);
        pl->timings[3] = nf;
        pl->timings[4] = ng;
        HIPCHK(hipEventElapsedTime(&ms, pl->ev[0], pl->ev.back()));
        pl->timings[5] = ms;
    }
    if (!finite) return fail(PR_ENONFINITE, "a defect norm is not finite (the iteration diverged or the input holds NaN/Inf)");
    return PR_OK;
}

int pr_set_kernel_variant(int32_t fine_variant, int32_t coarse_variant)
{
    if (fine_variant < 0 || fine_variant >= pr::fine_variant_count()) return fail(PR_EINVAL, "fine variant out of range");
    if (coarse_variant < 0 || coarse_variant >= pr::coarse_variant_count())
        return fail(PR_EINVAL, "coarse variant out of range");
    g_fine_forced = fine_variant;
    g_coarse_forced = coarse_variant;
    return PR_OK;
}

int pr_kernel_variant_count(int32_t which) { return which == 0 ? pr::fine_variant_count() : pr::coarse_variant_count(); }

const char *pr_kernel_variant_name(int32_t which, int32_t variant)
{
    if (variant == 0) return "auto";
    if (variant == 1) return which == 0 ? "rk4_unfused_reference" : "euler_unfused_reference";
    const VariantInfo *vi = which == 0 ? pr::fine_variant(variant) : pr::coarse_variant(variant);
    return vi ? vi->name : "invalid";
}

int pr_kernel_variant_info(int32_t which, int32_t variant, int32_t *dtype, int32_t *order, int32_t *tile_x,
                           int32_t *tile_y, int32_t *nxp, int32_t *steps, int32_t *nx_exact)
{
    const VariantInfo *vi = which == 0 ? pr::fine_variant(variant) : pr::coarse_variant(variant);
    if (!vi) return fail(PR_EINVAL, "no fused variant %d", variant);
    if (dtype) *dtype = vi->dtype;
    if (order) *order = vi->order;
    if (tile_x) *tile_x = vi->tx;
    if (tile_y) *tile_y = vi->ty;
    if (nxp) *nxp = vi->nxp;
    if (steps) *steps = vi->steps;
    if (nx_exact) *nx_exact = vi->rowx;
    return PR_OK;
}

int pr_sweep_kernel_variant(const pr_problem *prob, int32_t dtype, int32_t batch, int32_t which, int32_t *variant)
{
    int rc = validate_problem(prob, false);
    if (rc) return rc;
    if (dtype != PR_FP32 && dtype != PR_FP64) return fail(PR_EINVAL, "dtype must be PR_FP32 or PR_FP64");
    if (batch < 1 || (which != 0 && which != 1)) return fail(PR_EINVAL, "batch must be >= 1, which 0 or 1");
    pr_problem p = *prob;
    p.flags &= ~(PR_COARSEN_G | PR_CUBIC_INTERP);
    const Choice c = which == 0 ? pick_fine(p, dtype, batch) : pick_coarse(p, dtype, batch);
    if (c.v < 1) return fail(PR_EUNSUPPORTED, "no kernel variant for this problem");
    if (variant) *variant = c.v;
    return PR_OK;
}

size_t pr_autotune_workspace_bytes(const pr_problem *prob, int32_t dtype, int32_t batch)
{
    if (validate_problem(prob, false) || batch < 1 || (dtype != PR_FP32 && dtype != PR_FP64)) return 0;
    const size_t states = (size_t)batch * npts_of(*prob) * esize(dtype);
    return 2 * align256(states) + sweep_ws(*prob, dtype, batch, false);
}

int pr_autotune_save(const char *path)
{
    if (!path || !*path) return fail(PR_EINVAL, "path is NULL or empty");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    autoload_tune_cache_locked();
    return save_tune_cache_locked(path);
}

int pr_autotune_load(const char *path, int32_t *loaded)
{
    if (!path || !*path) return fail(PR_EINVAL, "path is NULL or empty");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    autoload_tune_cache_locked();
    int n = 0;
    const int rc = load_tune_cache_locked(path, &n);
    if (loaded) *loaded = n;
    return rc;
}

int pr_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    g_cache_loaded = true;   // an explicit clear also drops the environment's cache
    return PR_OK;
}

int pr_autotune(const pr_problem *prob, int32_t dtype, int32_t batch, int32_t which, void *ws, size_t ws_bytes,
                void *stream, int32_t *best_variant)
{
    int rc = validate_problem(prob, false);
    if (rc) return rc;
    if (which != 0 && which != 1) return fail(PR_EINVAL, "which must be 0 (fine) or 1 (coarse)");
    const size_t need = pr_autotune_workspace_bytes(prob, dtype, batch);
    if (!need) return fail(PR_EINVAL, "bad dtype or batch");
    if (!ws || ws_bytes < need) return fail(PR_ENOMEM, "workspace of %zu bytes < %zu needed", ws_bytes, need);
    rc = device_ready();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t states = (size_t)batch * npts_of(*prob) * esize(dtype);
    char *a = (char *)ws, *b = a + align256(states), *w = b + align256(states);
    const size_t wsb = sweep_ws(*prob, dtype, batch, false);
    HIPCHK(hipMemsetAsync(a, 0, states, s));
    pr_problem p = *prob;
    p.flags |= PR_ALLOW_UNSTABLE;  // zeros stay zeros; timing only
    p.flags &= ~(PR_COARSEN_G | PR_CUBIC_INTERP);
    std::vector<int64_t> st(batch, 0);
    const int saved_f = g_fine_forced, saved_c = g_coarse_forced, saved_b = g_bpc_forced;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    Choice bestc;
    const int nv = which == 0 ? pr::fine_variant_count() : pr::coarse_variant_count();
    static const int kBpc[] = {0, 1, 2, 4};   // 0: the resident blocks per compute unit
    for (int v = 2; v < nv && rc == PR_OK; ++v) {
        const bool ok = which == 0 ? fine_applicable(v, dtype, p.fine_order, p) : coarse_applicable(v, dtype, p);
        if (!ok) continue;
        for (int bpc : kBpc) {
            if (which == 0) g_fine_forced = v;
            else g_coarse_forced = v;
            g_bpc_forced = bpc;
            const int steps = which == 0 ? 6 : 8 * coarse_steps_per_launch(v);
            rc = sweep_common(&p, dtype, batch, a, b, st.data(), which == 0 ? 2 : 2 * coarse_steps_per_launch(v), w,
                              wsb, s, which == 0);
            if (rc) break;
            (void)hipEventRecord(e0, s);
            rc = sweep_common(&p, dtype, batch, a, b, st.data(), steps, w, wsb, s, which == 0);
            (void)hipEventRecord(e1, s);
            if (rc) break;
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const float per = ms / steps;
            if (per < best) {
                best = per;
                bestc.v = v;
                bestc.bpc = bpc;
            }
        }
    }
    g_fine_forced = saved_f;
    g_coarse_forced = saved_c;
    g_bpc_forced = saved_b;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (bestc.v < 2) return fail(PR_EUNSUPPORTED, "no fused variant applies");
    record_tuned(which, p, dtype, which == 0 ? p.fine_order : 0, batch, bestc);
    save_tune_cache_env();
    if (best_variant) *best_variant = bestc.v;
    return PR_OK;
}

int pr_plan_autotune(pr_plan *pl, void *stream, int32_t *fine_variant, int32_t *fine_blocks_per_cu,
                     int32_t *coarse_variant, int32_t *coarse_blocks_per_cu)
{
    if (!pl) return fail(PR_EINVAL, "plan is NULL");
    int rc = device_ready();
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const size_t es = esize(pl->dtype);
    // zero the sweep inputs of every slice and the coarse inputs: the timed
    // launches read them (times do not depend on the values)
    for (const auto &in : pl->inst) {
        HIPCHK(hipMemsetAsync(in.Ulo, 0, (size_t)(in.P + 1) * in.npts * es, s));
        if (in.Cin) HIPCHK(hipMemsetAsync(in.Cin, 0, (size_t)in.npts / 8 * es, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    static const int kBpc[] = {0, 1, 2, 4};   // 0: the resident blocks per compute unit
    std::vector<Choice> saved_f;
    for (const auto &g : pl->fgroups) saved_f.push_back(Choice{g.v, g.bpc});
    const Choice saved_g{pl->coarse_v, pl->coarse_bpc};
    // F candidates must apply to every instance of the group, G candidates
    // to every instance
    auto applies = [&](int which, int grp, int v) {
        for (int i = 0; i < pl->ninst; ++i) {
            const pr_problem &p = pl->probs[i];
            if (which == 0 && pl->inst_group[i] != grp) continue;
            const bool ok = which == 0 ? fine_applicable(v, pl->dtype, p.fine_order, p)
                                       : coarse_applicable(v, pl->dtype, coarse_grid(p));
            if (!ok) return false;
        }
        return true;
    };
    // time F step launches of one group over all its slices (iteration 0
    // table), and coarse chunks of the chain (slice 0 table) covering at
    // least 12 Euler steps; the figure compared is the time per step
    auto time_one = [&](int which, int grp, float *ms_out) -> int {
        int r = build_tables(pl);
        if (r) return r;
        const int S = which == 0 ? 1 : coarse_steps_per_launch(pl->coarse_v);
        const int launches = which == 0 ? 3 : std::max(3, (12 + S - 1) / S);
        for (int rep = 0; rep < 2; ++rep) {
            if (rep == 1) HIPCHK(hipEventRecord(e0, s));
            for (int t = 0; t < launches; ++t) {
                if (which == 0) {
                    const auto &g = pl->fgroups[grp];
                    if (g.active.empty() || g.active[0].empty()) break;
                    HIPCHK(pr::launch_fine_step(g.v, pl->dtype, pl->probs[0].fine_order, pl->fine_tab + g.off[0],
                                                g.cnt[0], g.active[0][0], 0, s));
                } else {
                    if (pl->coarse_cnt.empty() || !pl->coarse_cnt[0]) break;
                    HIPCHK(pr::launch_coarse_chunk(pl->coarse_v, pl->dtype, pl->coarse_tab, pl->coarse_cnt[0],
                                                   pl->coarse_blocks[0], 0, s));
                }
            }
        }
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        *ms_out = ms / (float)(launches * S);
        return PR_OK;
    };
    // one pass per F group, then G
    const int ngrp = (int)pl->fgroups.size();
    for (int pass = 0; pass <= ngrp && rc == PR_OK; ++pass) {
        const int which = pass < ngrp ? 0 : 1;
        const int grp = pass < ngrp ? pass : -1;
        if (which == 0 && pl->K == 0) continue;   // no fine sweep in the solve
        Choice best_c = which == 0 ? saved_f[grp] : saved_g;
        float best = 1e30f;
        const int nv = which == 0 ? pr::fine_variant_count() : pr::coarse_variant_count();
        for (int v = 2; v < nv && rc == PR_OK; ++v) {
            if (!applies(which, grp, v)) continue;
            const VariantInfo *vi = which == 0 ? pr::fine_variant(v) : pr::coarse_variant(v);
            if (which == 0 && vi->order != pl->probs[0].fine_order) continue;
            for (int bpc : kBpc) {
                if (which == 0) {
                    pl->fgroups[grp].v = v;
                    pl->fgroups[grp].bpc = bpc;
                } else {
                    pl->coarse_v = v;
                    pl->coarse_bpc = bpc;
                }
                float ms = 0;
                rc = time_one(which, grp, &ms);
                if (rc) break;
                if (ms < best) {
                    best = ms;
                    best_c = Choice{v, bpc};
                }
            }
        }
        if (which == 0) {
            pl->fgroups[grp].v = best_c.v;
            pl->fgroups[grp].bpc = best_c.bpc;
        } else {
            pl->coarse_v = best_c.v;
            pl->coarse_bpc = best_c.bpc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        for (int g = 0; g < ngrp; ++g) {
            pl->fgroups[g].v = saved_f[g].v;
            pl->fgroups[g].bpc = saved_f[g].bpc;
        }
        pl->coarse_v = saved_g.v;
        pl->coarse_bpc = saved_g.bpc;
    }
    if (!rc) {
        // remember the choices under the keys plan creation looks up: per
        // grid of a group, the batch of all slices of the instances with that
        // grid; G at the first instance's (coarse) grid and the instance count
        for (int g = 0; g < ngrp; ++g)
            for (int i : pl->fgroups[g].insts) {
                const pr_problem &pi = pl->probs[i];
                int batch = 0;
                for (int j = 0; j < pl->ninst; ++j)
                    if (pl->probs[j].n[0] == pi.n[0] && pl->probs[j].n[1] == pi.n[1] &&
                        pl->probs[j].n[2] == pi.n[2])
                        batch += pl->probs[j].P;
                record_tuned(0, pi, pl->dtype, pi.fine_order, batch, Choice{pl->fgroups[g].v, pl->fgroups[g].bpc});
            }
        record_tuned(1, coarse_grid(pl->probs[0]), pl->dtype, 0, pl->ninst, Choice{pl->coarse_v, pl->coarse_bpc});
        save_tune_cache_env();
    }
    int r2 = build_tables(pl);
    if (!rc) rc = r2;
    // a recorded graph holds the old launch shapes
    if (pl->exec) {
        (void)hipGraphExecDestroy(pl->exec);
        pl->exec = nullptr;
    }
    if (pl->graph_h) {
        (void)hipGraphDestroy(pl->graph_h);
        pl->graph_h = nullptr;
    }
    if (rc) return rc;
    const int pg = primary_group(pl);
    if (fine_variant) *fine_variant = pl->fgroups[pg].v;
    if (fine_blocks_per_cu) *fine_blocks_per_cu = pl->fgroups[pg].bpc;
    if (coarse_variant) *coarse_variant = pl->coarse_v;
    if (coarse_blocks_per_cu) *coarse_blocks_per_cu = pl->coarse_bpc;
    return PR_OK;
}

}  // extern "C"
