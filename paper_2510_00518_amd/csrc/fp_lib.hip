// libfp host runtime: context, loaders, launches of the rate kernels.
// Every entry point of include/fp.h except the host enumerator lives here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "fp.h"
#include "fp_kernels.h"

namespace {

// SI 2019 exact h, kB, e; CODATA 2018 atomic mass constant.  Internal units:
// energy amu*A^2/ps^2, action amu*A^2/ps.
constexpr double kPi = 3.14159265358979323846;
constexpr double kH = 6.62607015e-34;
constexpr double kKB = 1.380649e-23;
constexpr double kE = 1.602176634e-19;
constexpr double kAmu = 1.66053906660e-27;
const double kEnergyUnit = kAmu * 1e-20 / 1e-24;
const double kActionUnit = kAmu * 1e-20 / 1e-12;
const double kHbar = kH / (2.0 * kPi) / kActionUnit;
const double kBoltz = kKB / kEnergyUnit;
const double kEv = kE / kEnergyUnit;
const double kKappaUnit = kAmu * 1e-10 / 1e-36;  // amu*A/ps^3/K in W/(m K)

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t want) {
        if (want <= n && p) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            p = nullptr;
            n = 0;
            if (e != hipSuccess) return e;
        }
        size_t bytes = std::max<size_t>(want, 1) * sizeof(T);
        hipError_t e = hipMalloc(&p, bytes);
        if (e == hipSuccess) n = std::max<size_t>(want, 1);
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

struct IfcState {
    int32_t order = 0;
    int64_t n_terms = 0;
    int32_t n_groups = 0;
    std::vector<int32_t> atoms, cells;  // structure as loaded, to skip re-uploads
    DevBuf<double> raw, phi_s, scale;
    DevBuf<int32_t> perm, tmeta, tc, groups;
    void release() {
        raw.release(); phi_s.release(); scale.release();
        perm.release(); tmeta.release(); tc.release(); groups.release();
        order = 0; n_terms = 0; n_groups = 0;
        atoms.clear(); cells.clear();
    }
};

}  // namespace

struct fp_ctx {
    int device = 0;
    int n_cu = 256;
    std::string err;
    bool validate = false;
    // modes
    bool modes = false;
    int32_t mesh[3] = {0, 0, 0};
    int32_t nat = 0, nb = 0;
    int64_t nq = 0, n_modes = 0;
    int32_t L = 1;
    double volume = 0.0, floor_ = 0.0;
    bool have_vel = false;
    std::vector<double> masses;
    DevBuf<double> omega, vel;
    DevBuf<double2> evec, roots;
    IfcState ifc[2];  // order 3, order 4
    // per-call scratch (grow-only)
    DevBuf<double> occ, partial;
    DevBuf<fpk::RowInfo> rows;
    DevBuf<int64_t> row_units, unit_off;
    DevBuf<fpk::UnitDesc> units;
    DevBuf<double2> phit;
    int* flag = nullptr;
    // tuning knobs
    int32_t ppl = 2;
    int32_t blocks_per_cu = 2;
    // kernel timing
    bool profile = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;  // (order, (start, stop))
};

namespace {

fp_status fail(fp_ctx* c, fp_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(ctx, e_ == hipErrorOutOfMemory ? FP_ERR_NOMEM : FP_ERR_HIP, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                                 \
    } while (0)

int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

int64_t wrapi(int64_t x, int64_t n) { return ((x % n) + n) % n; }

fpk::ModeGeom geometry(const fp_ctx* c) {
    fpk::ModeGeom g;
    g.N0 = c->mesh[0];
    g.N1 = c->mesh[1];
    g.N2 = c->mesh[2];
    g.nb = c->nb;
    g.L = c->L;
    g.magic = (uint32_t)std::min<uint64_t>((uint64_t(1) << 32) / (uint64_t)c->L, 0xFFFFFFFFull);
    g.s0 = c->L / c->mesh[0];
    g.s1 = c->L / c->mesh[1];
    g.s2 = c->L / c->mesh[2];
    return g;
}

int grid_for(int64_t n, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

}  // namespace

extern "C" fp_status fp_create(fp_ctx** out, int32_t device) {
    if (!out) return FP_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FP_ERR_HIP;
    if (hipSetDevice(device) != hipSuccess) return FP_ERR_HIP;
    fp_ctx* c = new (std::nothrow) fp_ctx();
    if (!c) return FP_ERR_NOMEM;
    c->device = device;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->n_cu = ncu;
    const char* v = getenv("FP_VALIDATE");
    c->validate = v && v[0] == '1';
    if (hipMalloc(&c->flag, sizeof(int)) != hipSuccess) {
        delete c;
        return FP_ERR_NOMEM;
    }
    int zero = 0;
    if (hipMemcpy(c->flag, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(c->flag);
        delete c;
        return FP_ERR_HIP;
    }
    *out = c;
    return FP_OK;
}

extern "C" void fp_destroy(fp_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    c->omega.release(); c->vel.release(); c->evec.release(); c->roots.release();
    c->ifc[0].release(); c->ifc[1].release();
    c->occ.release(); c->partial.release(); c->rows.release(); c->row_units.release();
    c->unit_off.release(); c->units.release(); c->phit.release();
    if (c->flag) (void)hipFree(c->flag);
    for (auto& e : c->ev_used) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

extern "C" const char* fp_last_error(const fp_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" fp_status fp_set_knob(fp_ctx* c, const char* name, int64_t value) {
    if (!c || !name) return FP_ERR_ARG;
    if (!strcmp(name, "ppl")) {
        if (value < 1 || value > 64) return fail(c, FP_ERR_ARG, "ppl must be in [1, 64]");
        c->ppl = (int32_t)value;
    } else if (!strcmp(name, "blocks_per_cu")) {
        if (value < 1 || value > 16) return fail(c, FP_ERR_ARG, "blocks_per_cu must be in [1, 16]");
        c->blocks_per_cu = (int32_t)value;
    } else {
        return fail(c, FP_ERR_ARG, "unknown knob %s", name);
    }
    return FP_OK;
}

extern "C" fp_status fp_load_modes(fp_ctx* c, const int32_t mesh[3], int32_t n_atoms, const double lattice[9],
                                   const double* masses, const double* omega, const double* evec,
                                   const double* vel, double omega_floor) {
    if (!c) return FP_ERR_ARG;
    if (!mesh || !lattice || !masses || !omega || !evec) return fail(c, FP_ERR_ARG, "null argument");
    if (n_atoms < 1 || n_atoms > 32) return fail(c, FP_ERR_UNSUPPORTED, "n_atoms must be in [1, 32]");
    int64_t nq = 1, L = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh[d] < 1) return fail(c, FP_ERR_ARG, "mesh dimensions must be >= 1");
        nq *= mesh[d];
        L = L / gcd64(L, mesh[d]) * mesh[d];
    }
    const int32_t nb = 3 * n_atoms;
    if (nq * nb >= (int64_t(1) << 24)) return fail(c, FP_ERR_UNSUPPORTED, "more than 2^24 modes");
    if (L > fpk::kMaxRoots) return fail(c, FP_ERR_UNSUPPORTED, "lcm of the mesh dimensions exceeds 1024");
    for (int a = 0; a < n_atoms; ++a)
        if (!(masses[a] > 0.0) || !std::isfinite(masses[a])) return fail(c, FP_ERR_ARG, "masses must be > 0");
    const int64_t nm = nq * nb;
    for (int64_t g = 0; g < nm; ++g)
        if (!(omega[g] >= 0.0) || !std::isfinite(omega[g]))
            return fail(c, FP_ERR_ARG, "omega[%lld] is negative or not finite", (long long)g);
    for (int64_t i = 0; i < 2 * nm * nb; ++i)
        if (!std::isfinite(evec[i])) return fail(c, FP_ERR_ARG, "eigenvectors must be finite");
    if (!(omega_floor >= 0.0)) return fail(c, FP_ERR_ARG, "omega_floor must be >= 0");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, c->omega.ensure(nm));
    HIP_TRY(c, hipMemcpy(c->omega.p, omega, nm * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, c->evec.ensure(nm * nb));
    HIP_TRY(c, hipMemcpy(c->evec.p, evec, nm * nb * sizeof(double2), hipMemcpyHostToDevice));
    c->have_vel = vel != nullptr;
    if (vel) {
        HIP_TRY(c, c->vel.ensure(nm * 3));
        HIP_TRY(c, hipMemcpy(c->vel.p, vel, nm * 3 * sizeof(double), hipMemcpyHostToDevice));
    }
    std::vector<double2> roots((size_t)L);
    for (int64_t k = 0; k < L; ++k) {
        const double ang = 2.0 * kPi * (double)k / (double)L;
        roots[(size_t)k] = make_double2(std::cos(ang), std::sin(ang));
    }
    HIP_TRY(c, c->roots.ensure((size_t)L));
    HIP_TRY(c, hipMemcpy(c->roots.p, roots.data(), L * sizeof(double2), hipMemcpyHostToDevice));
    for (int d = 0; d < 3; ++d) c->mesh[d] = mesh[d];
    c->nat = n_atoms;
    c->nb = nb;
    c->nq = nq;
    c->n_modes = nm;
    c->L = (int32_t)L;
    c->floor_ = omega_floor;
    c->masses.assign(masses, masses + n_atoms);
    const double* A = lattice;
    c->volume = std::fabs(A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
                          A[2] * (A[3] * A[7] - A[4] * A[6]));
    c->ifc[0].release();
    c->ifc[1].release();
    c->modes = true;
    return FP_OK;
}

extern "C" fp_status fp_load_ifc(fp_ctx* c, int32_t order, int64_t n_terms, const int32_t* atoms,
                                 const int32_t* cells, const double* phi, int32_t phi_on_device, void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes must come first");
    if (order != 3 && order != 4) return fail(c, FP_ERR_ARG, "order must be 3 or 4");
    if (n_terms < 1 || n_terms > 4096) return fail(c, FP_ERR_UNSUPPORTED, "n_terms must be in [1, 4096]");
    if (!atoms || !cells || !phi) return fail(c, FP_ERR_ARG, "null argument");
    const int m = order;
    const int ncomp = m == 3 ? 27 : 81;
    for (int64_t i = 0; i < n_terms * m; ++i)
        if (atoms[i] < 0 || atoms[i] >= c->nat) return fail(c, FP_ERR_ARG, "atom index out of range");
    hipStream_t st = (hipStream_t)stream;
    IfcState& S = c->ifc[m - 3];
    HIP_TRY(c, hipSetDevice(c->device));
    const bool same = S.order == m && S.n_terms == n_terms &&
                      std::equal(atoms, atoms + n_terms * m, S.atoms.begin()) &&
                      std::equal(cells, cells + n_terms * (m - 1) * 3, S.cells.begin());
    if (!same) {
        // Structure: sort terms by the atoms of slots 1..m-1 (stable), build groups,
        // phase vectors and scale factors on the host.
        std::vector<int32_t> perm((size_t)n_terms);
        std::iota(perm.begin(), perm.end(), 0);
        auto key = [&](int32_t t) {
            int64_t k = 0;
            for (int r = 1; r < m; ++r) k = k * 64 + atoms[(int64_t)t * m + r];
            return k;
        };
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        std::vector<int32_t> tmeta((size_t)n_terms * 8, 0), tc((size_t)n_terms * 4, 0), groups;
        std::vector<double> scale((size_t)n_terms);
        const int64_t L = c->L;
        const int64_t sc[3] = {L / c->mesh[0], L / c->mesh[1], L / c->mesh[2]};
        for (int64_t i = 0; i < n_terms; ++i) {
            const int32_t t = perm[(size_t)i];
            const int32_t* at = atoms + (int64_t)t * m;
            const int32_t* ce = cells + (int64_t)t * (m - 1) * 3;
            const int32_t* Rl = ce + (m - 2) * 3;  // cell of the last slot
            double msc = 1.0;
            for (int r = 0; r < m; ++r) msc *= c->masses[at[r]];
            scale[(size_t)i] = kEv / std::sqrt(msc);
            tmeta[(size_t)i * 8 + 0] = at[0];
            for (int d = 0; d < 3; ++d) {
                // A = R1 - R_last, B = R2 - R_last (order 4), C = -R_last, scaled by L/N_d mod L
                tmeta[(size_t)i * 8 + 1 + d] = (int32_t)wrapi((int64_t)(ce[d] - Rl[d]) * sc[d], L);
                if (m == 4) tmeta[(size_t)i * 8 + 4 + d] = (int32_t)wrapi((int64_t)(ce[3 + d] - Rl[d]) * sc[d], L);
                tc[(size_t)i * 4 + d] = (int32_t)wrapi(-(int64_t)Rl[d] * sc[d], L);
            }
            const int64_t k = key(t);
            if (groups.empty() || key(perm[(size_t)groups[groups.size() - 8 + 3]]) != k) {
                const int32_t g[8] = {at[1], at[2], m == 4 ? at[3] : 0, (int32_t)i, (int32_t)i + 1, 0, 0, 0};
                groups.insert(groups.end(), g, g + 8);
            } else {
                groups[groups.size() - 8 + 4] = (int32_t)i + 1;
            }
        }
        HIP_TRY(c, hipStreamSynchronize(st));  // previous launches may still read the old tables
        HIP_TRY(c, S.perm.ensure((size_t)n_terms));
        HIP_TRY(c, S.scale.ensure((size_t)n_terms));
        HIP_TRY(c, S.tmeta.ensure(tmeta.size()));
        HIP_TRY(c, S.tc.ensure(tc.size()));
        HIP_TRY(c, S.groups.ensure(groups.size()));
        HIP_TRY(c, S.phi_s.ensure((size_t)n_terms * ncomp));
        HIP_TRY(c, hipMemcpy(S.perm.p, perm.data(), perm.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(S.scale.p, scale.data(), scale.size() * 8, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(S.tmeta.p, tmeta.data(), tmeta.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(S.tc.p, tc.data(), tc.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(S.groups.p, groups.data(), groups.size() * 4, hipMemcpyHostToDevice));
        S.order = m;
        S.n_terms = n_terms;
        S.n_groups = (int32_t)(groups.size() / 8);
        S.atoms.assign(atoms, atoms + n_terms * m);
        S.cells.assign(cells, cells + n_terms * (m - 1) * 3);
    }
    const double* src = phi;
    if (!phi_on_device) {
        HIP_TRY(c, S.raw.ensure((size_t)n_terms * ncomp));
        HIP_TRY(c, hipStreamSynchronize(st));
        HIP_TRY(c, hipMemcpy(S.raw.p, phi, (size_t)n_terms * ncomp * 8, hipMemcpyHostToDevice));
        src = S.raw.p;
    }
    hipLaunchKernelGGL(fpk::k_ifc_scale, dim3(grid_for(n_terms * ncomp)), dim3(256), 0, st, src, S.perm.p,
                       S.scale.p, n_terms, ncomp, S.phi_s.p);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

namespace {

fp_status run_rates(fp_ctx* c, int m, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                    double sigma, int32_t precision, double* gamma_out, double* wp_out, void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes must come first");
    IfcState& S = c->ifc[m - 3];
    if (S.order != m) return fail(c, FP_ERR_STATE, "force constants of order %d not loaded", m);
    const bool accumulate = (precision & FP_ACCUMULATE) != 0;
    precision &= ~FP_ACCUMULATE;
    if (precision != FP_FP64)
        return fail(c, FP_ERR_UNSUPPORTED, "only FP_FP64 is available for order %d", m);
    if (n_lists < 0 || n_lists > FP_MAX_LISTS || (n_lists > 0 && !lists))
        return fail(c, FP_ERR_ARG, "n_lists must be in [0, %d]", FP_MAX_LISTS);
    if (n_T < 1 || n_T > FP_MAX_T || !T_K) return fail(c, FP_ERR_ARG, "n_T must be in [1, %d]", FP_MAX_T);
    for (int i = 0; i < n_T; ++i)
        if (!(T_K[i] > 0.0) || !std::isfinite(T_K[i])) return fail(c, FP_ERR_ARG, "temperatures must be > 0");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(c, FP_ERR_ARG, "sigma must be > 0");
    fpk::ListsArg la;
    memset(&la, 0, sizeof la);
    la.n_lists = n_lists;
    int64_t total_rows = 0, n_units_max = 0;
    const int64_t unit = (int64_t)fpk::kWave * c->ppl;
    for (int l = 0; l < n_lists; ++l) {
        const fp_plist& P = lists[l];
        const bool ok_type = m == 3 ? (P.type == FP_3P || P.type == FP_3M)
                                    : (P.type == FP_4PP || P.type == FP_4PM || P.type == FP_4MM);
        if (!ok_type) return fail(c, FP_ERR_ARG, "list %d has type %d, not of order %d", l, P.type, m);
        if (P.n_rows < 0 || P.n_rec < 0) return fail(c, FP_ERR_ARG, "list %d: negative size", l);
        if (P.n_rows > 0 && (!P.row_mode || !P.row_off)) return fail(c, FP_ERR_ARG, "list %d: null row arrays", l);
        if (P.n_rec > 0 && !P.rec) return fail(c, FP_ERR_ARG, "list %d: null records", l);
        la.l[l].type = P.type;
        la.l[l].n_rows = P.n_rows;
        la.l[l].row_base = total_rows;
        la.l[l].n_rec = P.n_rec;
        la.l[l].row_mode = P.row_mode;
        la.l[l].row_off = P.row_off;
        la.l[l].rec = P.rec;
        total_rows += P.n_rows;
        n_units_max += (P.n_rec + unit - 1) / unit + P.n_rows;
    }
    la.total_rows = total_rows;
    if (total_rows > (int64_t(1) << 30)) return fail(c, FP_ERR_UNSUPPORTED, "too many rows");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nm = c->n_modes;
    const int ncomp = m == 3 ? 9 : 27;
    // scratch
    HIP_TRY(c, c->occ.ensure((size_t)n_T * nm));
    HIP_TRY(c, c->rows.ensure((size_t)std::max<int64_t>(total_rows, 1)));
    HIP_TRY(c, c->row_units.ensure((size_t)total_rows + 1));
    HIP_TRY(c, c->unit_off.ensure((size_t)total_rows + 1));
    HIP_TRY(c, c->units.ensure((size_t)std::max<int64_t>(n_units_max, 1)));
    HIP_TRY(c, c->partial.ensure((size_t)std::max<int64_t>(n_units_max, 1) * 2 * n_T));
    HIP_TRY(c, c->phit.ensure((size_t)std::max<int64_t>(total_rows, 1) * S.n_terms * ncomp));

    fpk::Temps tx;
    for (int i = 0; i < 8; ++i) tx.x[i] = i < n_T ? kHbar / (kBoltz * T_K[i]) : 0.0;
    // outputs are overwritten unless accumulating: zero them first
    if (gamma_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, gamma_out, n_T * nm, 0.0);
    if (wp_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, wp_out, n_T * nm, 0.0);
    if (total_rows == 0) {
        HIP_TRY(c, hipGetLastError());
        return FP_OK;
    }
    hipLaunchKernelGGL(fpk::k_occ, dim3(grid_for(n_T * nm)), dim3(256), 0, st, c->omega.p, nm, n_T, tx, c->floor_,
                       c->occ.p);
    hipLaunchKernelGGL(fpk::k_rows, dim3(grid_for(total_rows)), dim3(256), 0, st, la, nm, unit, c->rows.p,
                       c->row_units.p, c->flag);
    hipLaunchKernelGGL(fpk::k_scan, dim3(1), dim3(fpk::kBlock), 0, st, c->row_units.p, total_rows, c->unit_off.p);
    hipLaunchKernelGGL(fpk::k_units, dim3(grid_for(n_units_max)), dim3(256), 0, st, c->unit_off.p, total_rows,
                       c->rows.p, unit, n_units_max, c->units.p);
    const fpk::ModeGeom geo = geometry(c);
    const int64_t npre = total_rows * S.n_terms * ncomp;
    if (m == 3)
        hipLaunchKernelGGL(fpk::k_precontract<3>, dim3(grid_for(npre)), dim3(256), 0, st, c->rows.p, total_rows,
                           c->evec.p, c->roots.p, geo, S.phi_s.p, S.tmeta.p, S.tc.p, S.n_terms, c->phit.p);
    else
        hipLaunchKernelGGL(fpk::k_precontract<4>, dim3(grid_for(npre)), dim3(256), 0, st, c->rows.p, total_rows,
                           c->evec.p, c->roots.p, geo, S.phi_s.p, S.tmeta.p, S.tc.p, S.n_terms, c->phit.p);

    fpk::RatesArgs a;
    a.n_units = n_units_max;
    a.n_modes = nm;
    a.n_terms = (int32_t)S.n_terms;
    a.n_groups = S.n_groups;
    a.n_T = n_T;
    a.ppl = c->ppl;
    a.geo = geo;
    a.inv_sigma2 = 1.0 / (sigma * sigma);
    a.gnorm = 1.0 / (sigma * std::sqrt(kPi));
    const int64_t want_blocks = (n_units_max + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * c->blocks_per_cu, want_blocks);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    const int tsel = n_T == 1 ? 1 : (n_T <= 4 ? 4 : 8);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profile) {
        for (hipEvent_t* e : {&ev0, &ev1}) {
            if (!c->ev_pool.empty()) {
                *e = c->ev_pool.back();
                c->ev_pool.pop_back();
            } else {
                HIP_TRY(c, hipEventCreate(e));
            }
        }
        HIP_TRY(c, hipEventRecord(ev0, st));
    }
#define FP_LAUNCH(M, T)                                                                                         \
    hipLaunchKernelGGL((fpk::k_rates<M, T>), dim3((unsigned)nblk), dim3(fpk::kBlock), 0, st, c->omega.p, c->evec.p,   \
                       c->occ.p, c->roots.p, c->phit.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, \
                       c->flag, a)
    if (m == 3) {
        if (tsel == 1) FP_LAUNCH(3, 1); else if (tsel == 4) FP_LAUNCH(3, 4); else FP_LAUNCH(3, 8);
    } else {
        if (tsel == 1) FP_LAUNCH(4, 1); else if (tsel == 4) FP_LAUNCH(4, 4); else FP_LAUNCH(4, 8);
    }
#undef FP_LAUNCH
    if (c->profile) {
        HIP_TRY(c, hipEventRecord(ev1, st));
        c->ev_used.push_back({m, {ev0, ev1}});
    }
    const double N = (double)c->nq;
    const double pref = m == 3 ? kPi * kHbar / (4.0 * N) : kPi * kHbar * kHbar / (8.0 * N * N);
    const double wpref = m == 3 ? 1.0 / N : 1.0 / (N * N);
    for (int l = 0; l < n_lists; ++l) {
        if (la.l[l].n_rows == 0) continue;
        hipLaunchKernelGGL(fpk::k_finalize, dim3((unsigned)la.l[l].n_rows), dim3(fpk::kBlock), 0, st, c->partial.p,
                           c->unit_off.p, c->rows.p, la.l[l].row_base, n_T, pref, wpref, gamma_out, wp_out, nm);
    }
    HIP_TRY(c, hipGetLastError());
    if (c->validate) return fp_check(c, stream);
    return FP_OK;
}

}  // namespace

extern "C" fp_status fp_rates3(fp_ctx* c, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                               double sigma, int32_t precision, double* gamma_out, double* wp_out, void* stream) {
    return run_rates(c, 3, lists, n_lists, n_T, T_K, sigma, precision, gamma_out, wp_out, stream);
}

extern "C" fp_status fp_rates4(fp_ctx* c, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                               double sigma, int32_t precision, double* gamma_out, double* wp_out, void* stream) {
    return run_rates(c, 4, lists, n_lists, n_T, T_K, sigma, precision, gamma_out, wp_out, stream);
}

extern "C" fp_status fp_profile(fp_ctx* c, int32_t enable) {
    if (!c) return FP_ERR_ARG;
    for (auto& e : c->ev_used) {
        c->ev_pool.push_back(e.second.first);
        c->ev_pool.push_back(e.second.second);
    }
    c->ev_used.clear();
    c->profile = enable != 0;
    return FP_OK;
}

extern "C" fp_status fp_profile_read(fp_ctx* c, int32_t order, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches || (order != 3 && order != 4)) return FP_ERR_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    double tot = 0.0;
    int64_t n = 0;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> keep;
    for (auto& e : c->ev_used) {
        if (e.first != order) {
            keep.push_back(e);
            continue;
        }
        HIP_TRY(c, hipEventSynchronize(e.second.second));
        float ms = 0.0f;
        HIP_TRY(c, hipEventElapsedTime(&ms, e.second.first, e.second.second));
        tot += ms;
        ++n;
        c->ev_pool.push_back(e.second.first);
        c->ev_pool.push_back(e.second.second);
    }
    c->ev_used.swap(keep);
    *total_ms = tot;
    *launches = n;
    return FP_OK;
}

extern "C" fp_status fp_check(fp_ctx* c, void* stream) {
    if (!c) return FP_ERR_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipStreamSynchronize((hipStream_t)stream));
    int v = 0;
    HIP_TRY(c, hipMemcpy(&v, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    if (v) {
        int zero = 0;
        HIP_TRY(c, hipMemcpy(c->flag, &zero, sizeof(int), hipMemcpyHostToDevice));
        return fail(c, FP_ERR_RANGE, "a record or row mode lies outside the loaded mesh");
    }
    return FP_OK;
}

extern "C" fp_status fp_kappa_rta(fp_ctx* c, int32_t n_q1, const int32_t* q1, const double* q1_weight, int32_t n_T,
                                  const double* T_K, const double* gamma, double* kappa_out, double* dkappa_dgamma,
                                  void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes must come first");
    if (!c->have_vel) return fail(c, FP_ERR_STATE, "velocities were not loaded");
    if (n_q1 < 1 || n_q1 > c->nq || !q1 || !q1_weight || !gamma || !kappa_out)
        return fail(c, FP_ERR_ARG, "bad q1 list or null output");
    if (n_T < 1 || n_T > FP_MAX_T || !T_K) return fail(c, FP_ERR_ARG, "n_T must be in [1, %d]", FP_MAX_T);
    for (int i = 0; i < n_T; ++i)
        if (!(T_K[i] > 0.0)) return fail(c, FP_ERR_ARG, "temperatures must be > 0");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    fpk::Temps tx, pref;
    for (int i = 0; i < 8; ++i) {
        tx.x[i] = i < n_T ? kHbar / (kBoltz * T_K[i]) : 0.0;
        pref.x[i] = i < n_T ? kKappaUnit * kHbar * kHbar / ((double)c->nq * c->volume * kBoltz * T_K[i] * T_K[i])
                            : 0.0;
    }
    if (dkappa_dgamma)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * c->n_modes)), dim3(256), 0, st, dkappa_dgamma,
                           n_T * c->n_modes, 0.0);
    hipLaunchKernelGGL(fpk::k_kappa, dim3(n_T), dim3(fpk::kBlock), 0, st, q1, q1_weight, n_q1, c->nb, c->omega.p,
                       c->vel.p, gamma, c->n_modes, tx, pref, c->floor_, kappa_out, dkappa_dgamma, c->flag);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}
