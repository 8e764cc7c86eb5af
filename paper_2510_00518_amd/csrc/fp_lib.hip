// libfp host runtime: context, loaders, launches of the rate kernels.
// Every entry point of include/fp.h except the host enumerator lives here.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "fp.h"
#include "fp_kernels.h"
#include "fp_grad.h"
#include "fp_batched.h"
#include "fp_mixed.h"
#include "fp_fused.h"
#include "fp_probe.h"
#include "fp_enum_impl.h"

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
    bool borrowed = false;  // memory the buffer does not own (never freed or grown)
    hipError_t ensure(size_t want) {
        if (want <= n && p) return hipSuccess;
        if (borrowed) return hipErrorOutOfMemory;
        if (p) {
            // work queued on any stream may still read the old buffer
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return e;
            e = hipFree(p);
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
        if (p && !borrowed) (void)hipFree(p);
        p = nullptr;
        n = 0;
        borrowed = false;
    }
};

// Grow-only pinned host buffer (staging of streamed lists).
template <class T>
struct HostBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t want) {
        if (want <= n && p) return hipSuccess;
        release();
        const size_t m = std::max<size_t>(want, 1);
        hipError_t e = hipHostMalloc((void**)&p, m * sizeof(T), hipHostMallocDefault);
        if (e == hipSuccess) n = m;
        else p = nullptr;
        return e;
    }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
};

// One staging slot of the streaming executor: host and device copies of a chunk
// of lists, and the event that marks the end of the GPU work reading it.
struct StreamSlot {
    HostBuf<uint64_t> rec;
    HostBuf<int64_t> off;
    HostBuf<int32_t> mode;
    DevBuf<uint64_t> drec;
    DevBuf<int64_t> doff;
    DevBuf<int32_t> dmode;
    hipEvent_t done = nullptr;
    void release() {
        rec.release(); off.release(); mode.release();
        drec.release(); doff.release(); dmode.release();
        if (done) (void)hipEventDestroy(done);
        done = nullptr;
    }
};

struct IfcState {
    int32_t order = 0;
    int64_t n_terms = 0;
    int64_t n_keys = 0;  // phase keys (entries of the per-row tables)
    int32_t n_groups = 0;
    std::vector<int32_t> atoms, cells;  // structure as loaded, to skip re-uploads
    DevBuf<double> raw, phi_s, scale;
    // perm, scale, tc: per sorted term (tc = C scaled by L/N_d mod L, then a0);
    // tmeta: per phase key {first term, A, B, term count}; groups, pairs, kblk: over keys
    DevBuf<int32_t> perm, tmeta, tc, groups, pairs, kblk;
    int32_t n_pairs = 0;  // 16-key x 16-component tiles of the adjoint, within groups
    int32_t n_kblk = 0;   // 16-key K-blocks of the mixed-precision kernel, within groups
    // order 4, fused path: B-keys (runs of keys with the same partner atoms and B),
    // btab [n_bkeys][8] = {first key, 0, 0, 0, B (3), key count}; fgroups over
    // B-keys [n][8] = {atoms b, c, d, first B-key, end B-key, first K-step, 0, 0}
    DevBuf<int32_t> btab, fgroups;
    int32_t n_bkeys = 0, n_fgroups = 0, n_fks = 0;
    // order 4, fused path with the first partner folded per unit: pair groups over
    // the atoms of slots 2 and 3, each over "pkeys" (distinct B within the pair);
    // ptab [n_pkeys][8] = {first plist entry, entry count, 0, 0, B (3), 0},
    // plist [n][2] = {key, atom of slot 1}, pgroups [n][8] = {atoms c, d, first
    // pkey, end pkey, first K-step, 0, 0, 0}
    DevBuf<int32_t> ptab, plist, pgroups;
    int32_t n_pkeys = 0, n_pgroups = 0, n_pks = 0;
    void release() {
        raw.release(); phi_s.release(); scale.release();
        perm.release(); tmeta.release(); tc.release(); groups.release(); pairs.release(); kblk.release();
        btab.release(); fgroups.release(); ptab.release(); plist.release(); pgroups.release();
        order = 0; n_terms = 0; n_keys = 0; n_groups = 0; n_pairs = 0; n_kblk = 0;
        n_bkeys = 0; n_fgroups = 0; n_fks = 0; n_pkeys = 0; n_pgroups = 0; n_pks = 0;
        atoms.clear(); cells.clear();
    }
};

}  // namespace

// Fixed workspace of fp_rates4_noalloc: every device that runs the library
// holds its own copy until the process ends.  In host code `scratch` is a
// stand-in, not a device address; the address comes from hipGetSymbolAddress,
// taken once per device when the first context is created on it.
constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // per device, nullptr until looked up
}  // namespace

struct fp_ctx {
    int device = 0;
    void* scratch = nullptr;  // this device's address of `scratch`, or nullptr
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
    bool adaptive = false;      // per-process broadening (fp_set_broadening)
    double bfactor = 0.0;
    fp_broadening bro{};        // the setting behind proj, for the host enumerator
    DevBuf<double> proj;        // [n_modes][4] projections v . b_d / N_d and the frequency
    DevBuf<double> proj_max;    // [nq][4] largest |projection| over the branches of each q-point
    std::vector<double> masses;
    std::vector<double> h_omega, h_vel;  // host copies for the streaming executor's enumerator
    StreamSlot slot[2];
    DevBuf<double> omega, vel;
    DevBuf<double2> evec, roots;
    DevBuf<float2> evec32;  // FP32 copy of the eigenvectors for the mixed-precision contraction
    IfcState ifc[2];  // order 3, order 4
    // per-call scratch (grow-only)
    DevBuf<double> occ, partial;
    DevBuf<fpk::RowInfo> rows;
    DevBuf<int64_t> row_units, unit_off;
    DevBuf<fpk::UnitDesc> units;
    DevBuf<double2> phit;
    DevBuf<uint4> fsp;  // bf16 split planes of phit (mixed precision)
    DevBuf<double> gpart;
    DevBuf<double> gslab;       // first level of the partial-gradient reduction
    DevBuf<double> probe_out;   // results of the peak probes (one per thread)
    DevBuf<int64_t> sum_parts;  // per-block parts of the fused call's kept and tuple counts
    DevBuf<double> tune_out;  // scratch output of the autotuner's trial launches
    DevBuf<double2> hbuf;     // adjoint: c_p conj(V_p) per record of a range
    DevBuf<uint4> hdec;       // adjoint: each record's last partner and packed signed wavevectors
    DevBuf<double2> fold;     // fused FP64 path: one folded force-constant table per wave
    DevBuf<double> occt;      // fused form 2: occupations, temperature-fastest
    DevBuf<double> ev_val;    // three-phonon events: partner contributions per record
    DevBuf<int32_t> ev_key[2], ev_idx[2];  // their target modes and entries, unsorted and sorted
    DevBuf<unsigned char> ev_tmp;          // radix-sort workspace
    DevBuf<int64_t> unit_kept;  // fused enumeration: kept records per unit
    DevBuf<int64_t> unit_tup;   // fused enumeration: tuples with a kept record per unit
    DevBuf<int64_t> fused_cnt;  // last fused call: processes, tuples
    bool fused_done = false;
    int* flag = nullptr;
    // tuning knobs
    int32_t ppl = 2;
    int32_t blocks_per_cu = 0;  // 0: as many resident blocks as the kernel's occupancy allows
    int32_t variant = 6;        // order-4 contraction form: 0-3 per-process (k_rates), 4-7 tuple-batched
    int32_t grad_chunk = 4096;  // records per adjoint chunk (a multiple of 256)
    int64_t grad_records = int64_t(1) << 25;  // records per order-4 adjoint pass (bounds the h buffers: 1 GiB)
    int32_t fused_form = 2;     // FP64 form of fp_rates4_fused: 0 B-keys, 2 first partner folded
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

int ORDER_OF(int32_t type) { return type == FP_3P || type == FP_3M || type == FP_3E ? 3 : 4; }

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
    g.m_nb = 0xFFFFFFFFu / (uint32_t)c->nb;
    g.m_n2 = 0xFFFFFFFFu / (uint32_t)c->mesh[2];
    g.m_n12 = 0xFFFFFFFFu / (uint32_t)(c->mesh[1] * c->mesh[2]);
    return g;
}

int grid_for(int64_t n, int threads = 256) {
    int64_t b = (n + threads - 1) / threads;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

// Gaussian width of a call: `sigma` itself, or the floor of the per-process width
fpk::Broad make_broad(const fp_ctx* c, double sigma) {
    fpk::Broad b;
    b.inv_sigma2 = 1.0 / (sigma * sigma);
    b.gnorm = 1.0 / (sigma * std::sqrt(kPi));
    b.proj = c->adaptive ? c->proj.p : nullptr;
    b.factor = c->bfactor;
    b.floor_ = sigma;
    return b;
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
    {
        // the no-allocation workspace of this device (device current)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        void* ptr = device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
        if (!ptr) {
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
                ptr = nullptr;
                (void)hipGetLastError();
            } else if (device < kMaxDevices) {
                g_scratch_ptr[device] = ptr;
            }
        }
        c->scratch = ptr;
    }
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
    c->omega.release(); c->vel.release(); c->evec.release(); c->roots.release(); c->evec32.release();
    c->proj.release(); c->proj_max.release();
    c->ifc[0].release(); c->ifc[1].release();
    c->occ.release(); c->partial.release(); c->rows.release(); c->row_units.release();
    c->unit_off.release(); c->units.release(); c->phit.release(); c->gpart.release(); c->gslab.release(); c->probe_out.release(); c->sum_parts.release();
    c->fsp.release(); c->tune_out.release(); c->hbuf.release(); c->hdec.release(); c->fold.release(); c->occt.release();
    c->ev_val.release(); c->ev_key[0].release(); c->ev_key[1].release(); c->ev_idx[0].release();
    c->ev_idx[1].release(); c->ev_tmp.release(); c->unit_kept.release();
    c->unit_tup.release(); c->fused_cnt.release();
    c->slot[0].release(); c->slot[1].release();
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
        if (value < 0 || value > 16) return fail(c, FP_ERR_ARG, "blocks_per_cu must be in [0, 16]");
        c->blocks_per_cu = (int32_t)value;
    } else if (!strcmp(name, "grad_chunk")) {
        if (value < 256 || value > (1 << 22) || value % 256) return fail(c, FP_ERR_ARG, "grad_chunk: 256..2^22, multiple of 256");
        c->grad_chunk = (int32_t)value;
    } else if (!strcmp(name, "variant")) {
        if (value < 0 || value > 7) return fail(c, FP_ERR_ARG, "variant must be in [0, 7]");
        c->variant = (int32_t)value;
    } else if (!strcmp(name, "grad_records")) {
        if (value < 1024 || value > (int64_t(1) << 34)) return fail(c, FP_ERR_ARG, "grad_records: 1024..2^34");
        c->grad_records = value;
    } else if (!strcmp(name, "fused_form")) {
        if (value != 0 && value != 2) return fail(c, FP_ERR_ARG, "fused_form must be 0 or 2");
        c->fused_form = (int32_t)value;
    } else {
        return fail(c, FP_ERR_ARG, "unknown knob %s", name);
    }
    return FP_OK;
}

extern "C" fp_status fp_get_knob(fp_ctx* c, const char* name, int64_t* value) {
    if (!c || !name || !value) return FP_ERR_ARG;
    if (!strcmp(name, "ppl"))
        *value = c->ppl;
    else if (!strcmp(name, "blocks_per_cu"))
        *value = c->blocks_per_cu;
    else if (!strcmp(name, "grad_chunk"))
        *value = c->grad_chunk;
    else if (!strcmp(name, "variant"))
        *value = c->variant;
    else if (!strcmp(name, "fused_form"))
        *value = c->fused_form;
    else if (!strcmp(name, "grad_records"))
        *value = c->grad_records;
    else
        return fail(c, FP_ERR_ARG, "unknown knob %s", name);
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
    if (vel)
        for (int64_t i = 0; i < nm * 3; ++i)
            if (!std::isfinite(vel[i])) return fail(c, FP_ERR_ARG, "velocities must be finite");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, c->omega.ensure(nm));
    HIP_TRY(c, hipMemcpy(c->omega.p, omega, nm * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(c, c->evec.ensure(nm * nb));
    HIP_TRY(c, hipMemcpy(c->evec.p, evec, nm * nb * sizeof(double2), hipMemcpyHostToDevice));
    {
        std::vector<float2> e32((size_t)(nm * nb));
        for (int64_t i = 0; i < nm * nb; ++i) e32[(size_t)i] = make_float2((float)evec[2 * i], (float)evec[2 * i + 1]);
        HIP_TRY(c, c->evec32.ensure(nm * nb));
        HIP_TRY(c, hipMemcpy(c->evec32.p, e32.data(), e32.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
    c->have_vel = vel != nullptr;
    if (vel) {
        HIP_TRY(c, c->vel.ensure(nm * 3));
        HIP_TRY(c, hipMemcpy(c->vel.p, vel, nm * 3 * sizeof(double), hipMemcpyHostToDevice));
        c->h_vel.assign(vel, vel + nm * 3);
    } else {
        c->h_vel.clear();
    }
    c->h_omega.assign(omega, omega + nm);
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
    c->adaptive = false;
    c->modes = true;
    return FP_OK;
}

extern "C" fp_status fp_set_broadening(fp_ctx* c, const fp_broadening* b) {
    if (!c) return FP_ERR_ARG;
    if (!b || b->adaptive == 0) {
        c->adaptive = false;
        return FP_OK;
    }
    if (b->adaptive != 1) return fail(c, FP_ERR_ARG, "adaptive must be 0 or 1");
    if (!(b->factor > 0.0) || !std::isfinite(b->factor)) return fail(c, FP_ERR_ARG, "factor must be > 0");
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(b->recip[i])) return fail(c, FP_ERR_ARG, "reciprocal vectors must be finite");
    if (!c->modes || !c->have_vel) return fail(c, FP_ERR_STATE, "fp_load_modes with velocities must come first");
    fpk::RecipN r;
    for (int i = 0; i < 9; ++i) r.b[i] = b->recip[i];
    for (int d = 0; d < 3; ++d) r.inv_n[d] = 1.0 / (double)c->mesh[d];
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, c->proj.ensure((size_t)c->n_modes * 4));
    HIP_TRY(c, c->proj_max.ensure((size_t)c->nq * 4));
    hipLaunchKernelGGL(fpk::k_proj, dim3(grid_for(c->n_modes)), dim3(256), 0, nullptr, c->vel.p, c->omega.p,
                       c->n_modes, r, c->proj.p);
    hipLaunchKernelGGL(fpk::k_proj_max, dim3(grid_for(c->nq)), dim3(256), 0, nullptr, c->proj.p, (int64_t)c->nq,
                       (int)c->nb, c->proj_max.p);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipDeviceSynchronize());
    c->bfactor = b->factor;
    c->bro = *b;
    c->adaptive = true;
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
        // Structure.  The phase of term t in a process depends only on the
        // partner atoms and on the lattice vectors A = R1 - R_last (and
        // B = R2 - R_last for order 4) reduced modulo the mesh: exp(i Q.R) takes
        // the same value for R and R + N_d a_d.  Terms that agree in these (a
        // "phase key") share every phase, so once each is contracted with
        // e_lambda(a0) and exp(i q.C_t) per row, their tables add and the rate
        // kernels see one entry per key.  Terms are sorted by key (partner
        // atoms, then B, then A), keys are grouped by partner atoms.
        std::vector<int32_t> perm((size_t)n_terms);
        std::iota(perm.begin(), perm.end(), 0);
        const int64_t L = c->L;
        const int64_t sc[3] = {L / c->mesh[0], L / c->mesh[1], L / c->mesh[2]};
        auto phase_vec = [&](int32_t t, int r, int d) {  // (R_r - R_last)_d scaled by L/N_d, mod L; r = 1, 2
            const int32_t* ce = cells + (int64_t)t * (m - 1) * 3;
            const int32_t* Rl = ce + (m - 2) * 3;
            return (int32_t)wrapi((int64_t)(ce[(r - 1) * 3 + d] - Rl[d]) * sc[d], L);
        };
        auto key = [&](int32_t t) {
            std::vector<int64_t> k;
            for (int r = 1; r < m; ++r) k.push_back(atoms[(int64_t)t * m + r]);
            if (m == 4)
                for (int d = 0; d < 3; ++d) k.push_back(phase_vec(t, 2, d));
            for (int d = 0; d < 3; ++d) k.push_back(phase_vec(t, 1, d));
            return k;
        };
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return key(a) < key(b); });
        std::vector<int32_t> tmeta, tc((size_t)n_terms * 4, 0), groups;
        std::vector<double> scale((size_t)n_terms);
        std::vector<int64_t> prev;
        for (int64_t i = 0; i < n_terms; ++i) {
            const int32_t t = perm[(size_t)i];
            const int32_t* at = atoms + (int64_t)t * m;
            const int32_t* ce = cells + (int64_t)t * (m - 1) * 3;
            const int32_t* Rl = ce + (m - 2) * 3;  // cell of the last slot
            double msc = 1.0;
            for (int r = 0; r < m; ++r) msc *= c->masses[at[r]];
            scale[(size_t)i] = kEv / std::sqrt(msc);
            for (int d = 0; d < 3; ++d) tc[(size_t)i * 4 + d] = (int32_t)wrapi(-(int64_t)Rl[d] * sc[d], L);
            tc[(size_t)i * 4 + 3] = at[0];
            const std::vector<int64_t> k = key(t);
            if (i > 0 && k == prev) {
                ++tmeta[tmeta.size() - 1];  // one more term of this key
                continue;
            }
            prev = k;
            // a new key: {first sorted term, A (3), B (3), term count}
            const int32_t e[8] = {(int32_t)i, phase_vec(t, 1, 0), phase_vec(t, 1, 1), phase_vec(t, 1, 2),
                                  m == 4 ? phase_vec(t, 2, 0) : 0, m == 4 ? phase_vec(t, 2, 1) : 0,
                                  m == 4 ? phase_vec(t, 2, 2) : 0, 1};
            tmeta.insert(tmeta.end(), e, e + 8);
            const int32_t ki = (int32_t)(tmeta.size() / 8) - 1;
            // a group holds the keys of one partner-atom tuple, at most 16 of them
            // (larger ones are split), so one group's operands fit the rate
            // kernels' registers in one load
            const bool same_atoms = !groups.empty() && groups[groups.size() - 8] == at[1] &&
                                    groups[groups.size() - 7] == at[2] &&
                                    groups[groups.size() - 6] == (m == 4 ? at[3] : 0);
            if (same_atoms && groups[groups.size() - 8 + 4] - groups[groups.size() - 8 + 3] < 16) {
                groups[groups.size() - 8 + 4] = ki + 1;
            } else {
                const int32_t g[8] = {at[1], at[2], m == 4 ? at[3] : 0, ki, ki + 1, 0, 0, 0};
                groups.insert(groups.end(), g, g + 8);
            }
        }
        const int64_t n_keys = (int64_t)(tmeta.size() / 8);
        // K-blocks of the mixed-precision kernel: 16 consecutive keys of one group;
        // groups[g][5] is the group's first block, kblk[b] = {group, block within group}
        std::vector<int32_t> kblk;
        for (size_t g = 0; g + 8 <= groups.size(); g += 8) {
            groups[g + 5] = (int32_t)(kblk.size() / 2);
            for (int32_t tb = groups[g + 3], ks = 0; tb < groups[g + 4]; tb += 16, ++ks) {
                kblk.push_back((int32_t)(g / 8));
                kblk.push_back(ks);
            }
        }
        // adjoint tiles: 16 consecutive keys of one group x 16 components
        std::vector<int32_t> pairs;
        const int nc = m == 3 ? 9 : 27;
        for (size_t g = 0; g + 8 <= groups.size(); g += 8) {
            const int32_t t0 = groups[g + 3], t1 = groups[g + 4];
            for (int32_t tb = t0; tb < t1; tb += 16)
                for (int cb = 0; cb < nc; cb += 16) {
                    const int32_t e[4] = {(int32_t)(g / 8), tb, std::min<int32_t>(16, t1 - tb), cb};
                    pairs.insert(pairs.end(), e, e + 4);
                }
        }
        // B-keys of the fused path: within a unit (lambda, q') the phase
        // exp(i Q1.A) of every key is fixed, so the keys that share partner atoms
        // and B fold into one entry per unit and the per-tuple phase is exp(i Q2.B)
        std::vector<int32_t> btab, fgroups;
        int32_t n_fks = 0;
        if (m == 4) {
            for (size_t g = 0; g + 8 <= groups.size(); g += 8)
                for (int32_t k = groups[g + 3]; k < groups[g + 4]; ++k) {
                    const int32_t* e = tmeta.data() + (size_t)k * 8;
                    const bool same_b = !btab.empty() && e[4] == btab[btab.size() - 4] &&
                                        e[5] == btab[btab.size() - 3] && e[6] == btab[btab.size() - 2] &&
                                        k == btab[btab.size() - 8] + btab[btab.size() - 1] &&
                                        !fgroups.empty() && fgroups[fgroups.size() - 8] == groups[g] &&
                                        fgroups[fgroups.size() - 7] == groups[g + 1] &&
                                        fgroups[fgroups.size() - 6] == groups[g + 2];
                    if (same_b) {
                        ++btab[btab.size() - 1];
                        continue;
                    }
                    const int32_t b[8] = {k, 0, 0, 0, e[4], e[5], e[6], 1};
                    btab.insert(btab.end(), b, b + 8);
                    const int32_t bi = (int32_t)(btab.size() / 8) - 1;
                    const bool same_atoms = !fgroups.empty() && fgroups[fgroups.size() - 8] == groups[g] &&
                                            fgroups[fgroups.size() - 7] == groups[g + 1] &&
                                            fgroups[fgroups.size() - 6] == groups[g + 2];
                    if (same_atoms && fgroups[fgroups.size() - 4] - fgroups[fgroups.size() - 5] < 16) {
                        fgroups[fgroups.size() - 4] = bi + 1;
                    } else {
                        const int32_t f[8] = {groups[g], groups[g + 1], groups[g + 2], bi, bi + 1, 0, 0, 0};
                        fgroups.insert(fgroups.end(), f, f + 8);
                    }
                }
            for (size_t g = 0; g + 8 <= fgroups.size(); g += 8) {
                fgroups[g + 5] = n_fks;
                n_fks += (fgroups[g + 4] - fgroups[g + 3] + 3) / 4;
            }
        }
        // pair groups of the x-folded fused form: keys sorted by (atoms c, d; B;
        // atom b; key), runs of equal (c, d, B) form a pkey, at most 16 pkeys a group
        std::vector<int32_t> ptab, plist, pgroups;
        int32_t n_pks = 0;
        if (m == 4) {
            std::vector<std::array<int32_t, 6>> kk;  // c, d, B0, B1, B2, b ; then key
            std::vector<int32_t> kid;
            for (size_t g = 0; g + 8 <= groups.size(); g += 8)
                for (int32_t k = groups[g + 3]; k < groups[g + 4]; ++k) {
                    const int32_t* e = tmeta.data() + (size_t)k * 8;
                    kk.push_back({groups[g + 1], groups[g + 2], e[4], e[5], e[6], groups[g]});
                    kid.push_back(k);
                }
            std::vector<size_t> ord(kk.size());
            std::iota(ord.begin(), ord.end(), 0);
            std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
                return kk[x] != kk[y] ? kk[x] < kk[y] : kid[x] < kid[y];
            });
            for (size_t i = 0; i < ord.size(); ++i) {
                const auto& e = kk[ord[i]];
                const bool new_pkey = i == 0 || e[0] != kk[ord[i - 1]][0] || e[1] != kk[ord[i - 1]][1] ||
                                      e[2] != kk[ord[i - 1]][2] || e[3] != kk[ord[i - 1]][3] ||
                                      e[4] != kk[ord[i - 1]][4];
                if (new_pkey) {
                    const int32_t pe[8] = {(int32_t)(plist.size() / 2), 0, 0, 0, e[2], e[3], e[4], 0};
                    ptab.insert(ptab.end(), pe, pe + 8);
                    const int32_t pi = (int32_t)(ptab.size() / 8) - 1;
                    const bool same_pair = !pgroups.empty() && pgroups[pgroups.size() - 8] == e[0] &&
                                           pgroups[pgroups.size() - 7] == e[1];
                    if (same_pair && pgroups[pgroups.size() - 5] - pgroups[pgroups.size() - 6] < 16) {
                        pgroups[pgroups.size() - 5] = pi + 1;
                    } else {
                        const int32_t pg[8] = {e[0], e[1], pi, pi + 1, 0, 0, 0, 0};
                        pgroups.insert(pgroups.end(), pg, pg + 8);
                    }
                }
                ++ptab[ptab.size() - 8 + 1];
                plist.push_back(kid[ord[i]]);
                plist.push_back(e[5]);
            }
            for (size_t g = 0; g + 8 <= pgroups.size(); g += 8) {
                pgroups[g + 4] = n_pks;
                n_pks += (pgroups[g + 3] - pgroups[g + 2] + 3) / 4;
            }
        }
        HIP_TRY(c, hipStreamSynchronize(st));  // previous launches may still read the old tables
        if (m == 4) {
            HIP_TRY(c, S.ptab.ensure(ptab.size()));
            HIP_TRY(c, hipMemcpy(S.ptab.p, ptab.data(), ptab.size() * 4, hipMemcpyHostToDevice));
            HIP_TRY(c, S.plist.ensure(plist.size()));
            HIP_TRY(c, hipMemcpy(S.plist.p, plist.data(), plist.size() * 4, hipMemcpyHostToDevice));
            HIP_TRY(c, S.pgroups.ensure(pgroups.size()));
            HIP_TRY(c, hipMemcpy(S.pgroups.p, pgroups.data(), pgroups.size() * 4, hipMemcpyHostToDevice));
        }
        S.n_pkeys = (int32_t)(ptab.size() / 8);
        S.n_pgroups = (int32_t)(pgroups.size() / 8);
        S.n_pks = n_pks;
        if (m == 4) {
            HIP_TRY(c, S.btab.ensure(btab.size()));
            HIP_TRY(c, hipMemcpy(S.btab.p, btab.data(), btab.size() * 4, hipMemcpyHostToDevice));
            HIP_TRY(c, S.fgroups.ensure(fgroups.size()));
            HIP_TRY(c, hipMemcpy(S.fgroups.p, fgroups.data(), fgroups.size() * 4, hipMemcpyHostToDevice));
        }
        S.n_bkeys = (int32_t)(btab.size() / 8);
        S.n_fgroups = (int32_t)(fgroups.size() / 8);
        S.n_fks = n_fks;
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
        HIP_TRY(c, S.pairs.ensure(pairs.size()));
        HIP_TRY(c, hipMemcpy(S.pairs.p, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice));
        S.n_pairs = (int32_t)(pairs.size() / 4);
        HIP_TRY(c, S.kblk.ensure(kblk.size()));
        HIP_TRY(c, hipMemcpy(S.kblk.p, kblk.data(), kblk.size() * 4, hipMemcpyHostToDevice));
        S.n_kblk = (int32_t)(kblk.size() / 2);
        S.order = m;
        S.n_terms = n_terms;
        S.n_keys = n_keys;
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

extern "C" fp_status fp_ifc_info(fp_ctx* c, int32_t order, int64_t out[5]) {
    if (!c) return FP_ERR_ARG;
    if (!out || (order != 3 && order != 4)) return fail(c, FP_ERR_ARG, "out must be non-null, order 3 or 4");
    const IfcState& S = c->ifc[order - 3];
    if (S.order != order) return fail(c, FP_ERR_STATE, "force constants of order %d not loaded", order);
    out[0] = S.n_terms;
    out[1] = S.n_keys;
    out[2] = S.n_groups;
    out[3] = S.n_pkeys;
    out[4] = S.n_pgroups;
    return FP_OK;
}

namespace {

// order-4 contraction variants: (form, processes per lane)
struct Variant {
    int ct, np;
};
// 4-7: tuple-batched (two records per lane; one; two with 24-tuple batches at 3 blocks per CU; three)
constexpr Variant kVariants[8] = {{0, 1}, {1, 1}, {1, 2}, {0, 2}, {2, 2}, {2, 1}, {2, 2}, {2, 3}};

// records per lane of the tuple-batched forms (units of 64 x this many records)
inline int batched_br(int variant) { return variant == 5 ? 1 : (variant == 7 ? 3 : fpk::kBR); }

template <int M, int T, int CT, int NP>
fp_status launch_rates(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S) {
    auto kern = fpk::k_rates<M, T, CT, NP, 1>;
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, 0));
    if (occ < 1) occ = 1;
    const int bpc = c->blocks_per_cu > 0 ? std::min(c->blocks_per_cu, occ) : occ;
    const int64_t want = (n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * bpc, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), 0, st, c->omega.p, c->evec.p, c->occ.p,
                       c->roots.p, c->phit.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, c->flag, a);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

template <int T>
fp_status launch_mixed(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S) {
    auto kern = fpk::k_rates4m<T, false>;
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, 0));
    if (occ < 1) occ = 1;
    const int bpc = c->blocks_per_cu > 0 ? std::min(c->blocks_per_cu, occ) : occ;
    const int64_t want = (n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * bpc, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), 0, st, c->omega.p, c->evec32.p, c->occ.p,
                       c->roots.p, c->fsp.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, c->flag, a,
                       S.n_kblk, (const double*)nullptr, 0.0, (double2*)nullptr, (uint4*)nullptr);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

// First pass of the mixed-precision order-4 adjoint (units of 128 records).
template <int T>
fp_status launch_mixed_h(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S,
                         const double* dldg, double pref) {
    auto kern = fpk::k_rates4m<T, true>;
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, 0));
    if (occ < 1) occ = 1;
    const int64_t want = (n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * occ, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), 0, st, c->omega.p, c->evec32.p, c->occ.p,
                       c->roots.p, c->fsp.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, c->flag, a,
                       S.n_kblk, dldg, pref, c->hbuf.p, c->hdec.p);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

template <int T, int BR, int TB, int OCC>
fp_status launch_batched(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S) {
    auto kern = fpk::k_rates4b<T, false, BR, TB, OCC>;
    const size_t shm = fpk::tb_dyn_lds(c->L, S.n_keys);
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, shm));
    if (occ < 1) occ = 1;
    const int bpc = c->blocks_per_cu > 0 ? std::min(c->blocks_per_cu, occ) : occ;
    const int64_t want = (n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * bpc, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), shm, st, c->omega.p, c->evec.p, c->occ.p,
                       c->roots.p, c->phit.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, c->flag, a,
                       (const double*)nullptr, 0.0, (double2*)nullptr, (uint4*)nullptr);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

// First half of the order-4 adjoint: h_p = c_p conj(V_p) per record, by the
// tuple-batched kernel over units of 128 records (24-tuple batches, three
// resident blocks per CU).
template <int T>
fp_status launch_batched_h(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S,
                           const double* dldg, double pref) {
    auto kern = fpk::k_rates4b<T, true, 2, 24, 3>;
    const size_t shm = fpk::tb_dyn_lds(c->L, S.n_keys);
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, shm));
    if (occ < 1) occ = 1;
    const int64_t want = (n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * occ, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), shm, st, c->omega.p, c->evec.p, c->occ.p,
                       c->roots.p, c->phit.p, S.tmeta.p, S.groups.p, c->rows.p, c->units.p, c->partial.p, c->flag, a,
                       dldg, pref, c->hbuf.p, c->hdec.p);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

template <int M, int T>
fp_status launch_variant(fp_ctx* c, hipStream_t st, int64_t n_units, const fpk::RatesArgs& a, const IfcState& S) {
    if (M == 3) return launch_rates<3, T, 0, 1>(c, st, n_units, a, S);
    switch (c->variant) {
        case 4: return launch_batched<T, fpk::kBR, fpk::kTB, 2>(c, st, n_units, a, S);
        case 5: return launch_batched<T, 1, 16, 2>(c, st, n_units, a, S);
        case 6: return launch_batched<T, fpk::kBR, 24, 3>(c, st, n_units, a, S);
        case 7: return launch_batched<T, 3, 32, 2>(c, st, n_units, a, S);
        case 1: return launch_rates<4, T, 1, 1>(c, st, n_units, a, S);
        case 2: return launch_rates<4, T, 1, 2>(c, st, n_units, a, S);
        case 3: return launch_rates<4, T, 0, 2>(c, st, n_units, a, S);
        default: return launch_rates<4, T, 0, 1>(c, st, n_units, a, S);
    }
}

double rate_prefactor(const fp_ctx* c, int m) {
    const double N = (double)c->nq;
    return m == 3 ? kPi * kHbar / (4.0 * N) : kPi * kHbar * kHbar / (8.0 * N * N);
}

// Checks shared by the rate and adjoint calls.
fp_status check_common(fp_ctx* c, int n_lists, const fp_plist* lists, int32_t n_T, const double* T_K, double sigma) {
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes must come first");
    if (n_lists < 0 || n_lists > FP_MAX_LISTS || (n_lists > 0 && !lists))
        return fail(c, FP_ERR_ARG, "n_lists must be in [0, %d]", FP_MAX_LISTS);
    if (n_T < 1 || n_T > FP_MAX_T || !T_K) return fail(c, FP_ERR_ARG, "n_T must be in [1, %d]", FP_MAX_T);
    for (int i = 0; i < n_T; ++i)
        if (!(T_K[i] > 0.0) || !std::isfinite(T_K[i])) return fail(c, FP_ERR_ARG, "temperatures must be > 0");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(c, FP_ERR_ARG, "sigma must be > 0");
    for (int l = 0; l < n_lists; ++l) {
        const fp_plist& P = lists[l];
        if (P.type < FP_3P || P.type > FP_3E) return fail(c, FP_ERR_ARG, "list %d has unknown type %d", l, P.type);
        if (P.n_rows < 0 || P.n_rec < 0) return fail(c, FP_ERR_ARG, "list %d: negative size", l);
        if (P.n_rows > 0 && (!P.row_mode || !P.row_off)) return fail(c, FP_ERR_ARG, "list %d: null row arrays", l);
        if (P.n_rec > 0 && !P.rec) return fail(c, FP_ERR_ARG, "list %d: null records", l);
    }
    return FP_OK;
}

struct Prepared {
    fpk::ListsArg la;
    int64_t total_rows = 0, n_units = 0;
    fpk::ModeGeom geo;
};

// Per-call device tables for the lists of order m (sel[] picks them): Bose
// table, row table, work units of `unit` records, and the pre-contracted
// force constants of every row.
fp_status prepare(fp_ctx* c, int m, const fp_plist* lists, const std::vector<int>& sel, int32_t n_T,
                  const double* T_K, int64_t unit, hipStream_t st, Prepared* pp,
                  const std::vector<int64_t>* rec_shift = nullptr) {
    IfcState& S = c->ifc[m - 3];
    fpk::ListsArg& la = pp->la;
    memset(&la, 0, sizeof la);
    la.n_lists = (int32_t)sel.size();
    int64_t total_rows = 0, n_units = 0, rec_base = 0;
    for (size_t k = 0; k < sel.size(); ++k) {
        const fp_plist& P = lists[sel[k]];
        la.l[k].rec_base = rec_base;
        rec_base += P.n_rec;
        la.l[k].type = P.type;
        la.l[k].n_rows = P.n_rows;
        la.l[k].row_base = total_rows;
        la.l[k].n_rec = P.n_rec;
        la.l[k].row_mode = P.row_mode;
        la.l[k].row_off = P.row_off;
        la.l[k].rec = P.rec;
        la.l[k].rec_shift = rec_shift ? (*rec_shift)[k] : 0;
        total_rows += P.n_rows;
        n_units += (P.n_rec + unit - 1) / unit + P.n_rows;
    }
    la.total_rows = total_rows;
    pp->total_rows = total_rows;
    pp->n_units = n_units;
    pp->geo = geometry(c);
    if (total_rows > (int64_t(1) << 30)) return fail(c, FP_ERR_UNSUPPORTED, "too many rows");
    if (total_rows == 0) return FP_OK;
    const int64_t nm = c->n_modes;
    const int ncomp = m == 3 ? 9 : 27;
    HIP_TRY(c, c->occ.ensure((size_t)n_T * nm));
    HIP_TRY(c, c->rows.ensure((size_t)total_rows));
    HIP_TRY(c, c->row_units.ensure((size_t)total_rows + 1));
    HIP_TRY(c, c->unit_off.ensure((size_t)total_rows + 1));
    HIP_TRY(c, c->units.ensure((size_t)std::max<int64_t>(n_units, 1)));
    HIP_TRY(c, c->phit.ensure((size_t)total_rows * S.n_keys * ncomp));
    fpk::Temps tx;
    for (int i = 0; i < 8; ++i) tx.x[i] = i < n_T ? kHbar / (kBoltz * T_K[i]) : 0.0;
    hipLaunchKernelGGL(fpk::k_occ, dim3(grid_for(n_T * nm)), dim3(256), 0, st, c->omega.p, nm, n_T, tx, c->floor_,
                       c->occ.p);
    hipLaunchKernelGGL(fpk::k_rows, dim3(grid_for(total_rows)), dim3(256), 0, st, la, nm, unit, c->rows.p,
                       c->row_units.p, c->flag);
    hipLaunchKernelGGL(fpk::k_scan, dim3(1), dim3(fpk::kBlock), 0, st, c->row_units.p, total_rows, c->unit_off.p);
    hipLaunchKernelGGL(fpk::k_units, dim3(grid_for(n_units)), dim3(256), 0, st, c->unit_off.p, total_rows, c->rows.p,
                       unit, n_units, c->units.p);
    const int64_t npre = total_rows * S.n_keys * ncomp;
    if (m == 3)
        hipLaunchKernelGGL(fpk::k_precontract<3>, dim3(grid_for(npre)), dim3(256), 0, st, c->rows.p, total_rows,
                           c->evec.p, c->roots.p, pp->geo, S.phi_s.p, S.tmeta.p, S.tc.p, S.n_keys, c->phit.p);
    else
        hipLaunchKernelGGL(fpk::k_precontract<4>, dim3(grid_for(npre)), dim3(256), 0, st, c->rows.p, total_rows,
                           c->evec.p, c->roots.p, pp->geo, S.phi_s.p, S.tmeta.p, S.tc.p, S.n_keys, c->phit.p);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

fp_status timer_start(fp_ctx* c, hipStream_t st, hipEvent_t* ev0, hipEvent_t* ev1) {
    *ev0 = *ev1 = nullptr;
    if (!c->profile) return FP_OK;
    for (hipEvent_t* e : {ev0, ev1}) {
        if (!c->ev_pool.empty()) {
            *e = c->ev_pool.back();
            c->ev_pool.pop_back();
        } else {
            HIP_TRY(c, hipEventCreate(e));
        }
    }
    HIP_TRY(c, hipEventRecord(*ev0, st));
    return FP_OK;
}

fp_status timer_stop(fp_ctx* c, hipStream_t st, int tag, hipEvent_t ev0, hipEvent_t ev1) {
    if (!c->profile) return FP_OK;
    HIP_TRY(c, hipEventRecord(ev1, st));
    c->ev_used.push_back({tag, {ev0, ev1}});
    return FP_OK;
}

// Records per lane of a work unit (units hold 64 times this many records): the
// tuple-batched and mixed kernels fix it, the per-process forms take the knob.
int64_t unit_ppl(const fp_ctx* c, int m, bool mixed) {
    const int np = m == 3 ? 1 : kVariants[c->variant].np;
    return mixed ? fpk::kBR : (m == 4 && c->variant >= 4) ? batched_br(c->variant) : (c->ppl + np - 1) / np * np;
}

fp_status run_rates(fp_ctx* c, int m, const fp_plist* lists, int32_t n_lists, int32_t n_T, const double* T_K,
                    double sigma, int32_t precision, double* gamma_out, double* wp_out, void* stream) {
    if (!c) return FP_ERR_ARG;
    fp_status cs = check_common(c, n_lists, lists, n_T, T_K, sigma);
    if (cs != FP_OK) return cs;
    IfcState& S = c->ifc[m - 3];
    if (S.order != m) return fail(c, FP_ERR_STATE, "force constants of order %d not loaded", m);
    const bool accumulate = (precision & FP_ACCUMULATE) != 0;
    precision &= ~FP_ACCUMULATE;
    if (precision != FP_FP64 && precision != FP_MIXED) return fail(c, FP_ERR_ARG, "unknown precision %d", precision);
    // order 3 is a negligible share of the work and always runs in FP64
    const bool mixed = precision == FP_MIXED && m == 4;
    std::vector<int> sel;
    for (int l = 0; l < n_lists; ++l) {
        if (ORDER_OF(lists[l].type) != m)
            return fail(c, FP_ERR_ARG, "list %d has type %d, not of order %d", l, lists[l].type, m);
        if (lists[l].type == FP_3E && c->adaptive)
            return fail(c, FP_ERR_UNSUPPORTED, "event lists take the fixed width only");
        sel.push_back(l);
    }
    const int64_t ppl = unit_ppl(c, m, mixed);
    const int64_t unit = (int64_t)fpk::kWave * ppl;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nm = c->n_modes;
    // outputs are overwritten unless accumulating: zero them first
    if (gamma_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, gamma_out, n_T * nm, 0.0);
    if (wp_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, wp_out, n_T * nm, 0.0);
    Prepared pp;
    fp_status ps = prepare(c, m, lists, sel, n_T, T_K, unit, st, &pp);
    if (ps != FP_OK) return ps;
    if (pp.total_rows == 0) {
        HIP_TRY(c, hipGetLastError());
        return FP_OK;
    }
    HIP_TRY(c, c->partial.ensure((size_t)std::max<int64_t>(pp.n_units, 1) * 2 * n_T));
    fpk::RatesArgs a;
    a.n_units = pp.n_units;
    a.n_modes = nm;
    a.n_keys = (int32_t)S.n_keys;
    a.n_groups = S.n_groups;
    a.n_T = n_T;
    a.ppl = (int32_t)ppl;
    a.geo = pp.geo;
    a.br = make_broad(c, sigma);
    a.pref = rate_prefactor(c, m);
    a.wpref = m == 3 ? 1.0 / (double)c->nq : 1.0 / ((double)c->nq * (double)c->nq);
    a.ev_val = nullptr;
    a.ev_key = nullptr;
    // three-phonon event lists: per-record partner contributions, reduced per mode
    // in a fixed order after the row sums (k_event_reduce)
    bool events = false;
    int64_t n_all = 0;  // records of the call
    for (int l : sel) {
        events = events || lists[l].type == FP_3E;
        n_all += lists[l].n_rec;
    }
    if (events) {
        HIP_TRY(c, c->ev_val.ensure((size_t)std::max<int64_t>(2 * n_all * 2 * n_T, 1)));
        for (int i = 0; i < 2; ++i) {
            HIP_TRY(c, c->ev_key[i].ensure((size_t)std::max<int64_t>(2 * n_all, 1)));
            HIP_TRY(c, c->ev_idx[i].ensure((size_t)std::max<int64_t>(2 * n_all, 1)));
        }
        hipLaunchKernelGGL(fpk::k_fill_i32, dim3(grid_for(2 * n_all)), dim3(256), 0, st, c->ev_key[0].p, 2 * n_all,
                           (int32_t)0x7FFFFFFF);
        a.ev_val = c->ev_val.p;
        a.ev_key = c->ev_key[0].p;
    }
    const int tsel = n_T == 1 ? 1 : (n_T <= 4 ? 4 : 8);
    if (mixed) {
        const int64_t nf = pp.total_rows * S.n_kblk * 4 * fpk::kWave;
        HIP_TRY(c, c->fsp.ensure((size_t)std::max<int64_t>(nf * 3, 1)));
        hipLaunchKernelGGL(fpk::k_split_phit, dim3(grid_for(nf)), dim3(256), 0, st, pp.total_rows, c->phit.p,
                           S.groups.p, S.kblk.p, S.n_kblk, (int32_t)S.n_keys, c->fsp.p);
        HIP_TRY(c, hipGetLastError());
    }
    hipEvent_t ev0, ev1;
    fp_status ts = timer_start(c, st, &ev0, &ev1);
    if (ts != FP_OK) return ts;
    fp_status ls;
    if (mixed)
        ls = tsel == 1 ? launch_mixed<1>(c, st, pp.n_units, a, S)
                       : (tsel == 4 ? launch_mixed<4>(c, st, pp.n_units, a, S) : launch_mixed<8>(c, st, pp.n_units, a, S));
    else if (m == 3)
        ls = tsel == 1 ? launch_variant<3, 1>(c, st, pp.n_units, a, S)
                       : (tsel == 4 ? launch_variant<3, 4>(c, st, pp.n_units, a, S)
                                    : launch_variant<3, 8>(c, st, pp.n_units, a, S));
    else
        ls = tsel == 1 ? launch_variant<4, 1>(c, st, pp.n_units, a, S)
                       : (tsel == 4 ? launch_variant<4, 4>(c, st, pp.n_units, a, S)
                                    : launch_variant<4, 8>(c, st, pp.n_units, a, S));
    if (ls != FP_OK) return ls;
    ts = timer_stop(c, st, mixed ? 24 : m, ev0, ev1);
    if (ts != FP_OK) return ts;
    const double pref = rate_prefactor(c, m);
    const double wpref = m == 3 ? 1.0 / (double)c->nq : 1.0 / ((double)c->nq * (double)c->nq);
    for (int k = 0; k < pp.la.n_lists; ++k) {
        if (pp.la.l[k].n_rows == 0) continue;
        hipLaunchKernelGGL(fpk::k_finalize, dim3((unsigned)pp.la.l[k].n_rows), dim3(fpk::kBlock), 0, st,
                           c->partial.p, c->unit_off.p, c->rows.p, pp.la.l[k].row_base, n_T, pref, wpref, gamma_out,
                           wp_out, nm);
    }
    if (events && n_all > 0) {
        // stable sort of (target mode, entry) pairs, then one ordered sum per mode
        const int n = (int)(2 * n_all);
        if (2 * n_all > INT32_MAX) return fail(c, FP_ERR_UNSUPPORTED, "too many event records");
        hipLaunchKernelGGL(fpk::k_iota_i32, dim3(grid_for(n)), dim3(256), 0, st, c->ev_idx[0].p, (int64_t)n);
        size_t bytes = 0;
        HIP_TRY(c, hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, c->ev_key[0].p, c->ev_key[1].p, c->ev_idx[0].p,
                                                      c->ev_idx[1].p, n, 0, 32, st));
        HIP_TRY(c, c->ev_tmp.ensure(std::max<size_t>(bytes, 1)));
        HIP_TRY(c, hipcub::DeviceRadixSort::SortPairs(c->ev_tmp.p, bytes, c->ev_key[0].p, c->ev_key[1].p,
                                                      c->ev_idx[0].p, c->ev_idx[1].p, n, 0, 32, st));
        hipLaunchKernelGGL(fpk::k_event_reduce, dim3(grid_for(nm)), dim3(256), 0, st, c->ev_key[1].p, c->ev_idx[1].p,
                           (int64_t)n, c->ev_val.p, n_T, gamma_out, wp_out, nm);
    }
    HIP_TRY(c, hipGetLastError());
    if (c->validate) return fp_check(c, stream);
    return FP_OK;
}

// dphi (+)= the sum of n_parts partial gradients in gpart, in part order; above
// two slabs, slabs of kSlab parts are summed first (deterministic either way).
fp_status reduce_partials(fp_ctx* c, hipStream_t st, int64_t n_parts, const IfcState& S, int32_t ncomp,
                          bool accumulate, double* dphi) {
    const int64_t per = (int64_t)S.n_terms * ncomp;
    const double* src = c->gpart.p;
    int64_t n = n_parts;
    if (n_parts > 2 * fpk::kSlab) {
        const int64_t n_slabs = (n_parts + fpk::kSlab - 1) / fpk::kSlab;
        HIP_TRY(c, c->gslab.ensure((size_t)(n_slabs * per)));
        hipLaunchKernelGGL(fpk::k_grad_slab, dim3(grid_for(n_slabs * per)), dim3(256), 0, st, c->gpart.p, n_parts, per,
                           c->gslab.p);
        src = c->gslab.p;
        n = n_slabs;
    }
    hipLaunchKernelGGL(fpk::k_grad_reduce, dim3(grid_for(per)), dim3(256), 0, st, src, n, S.n_terms, ncomp,
                       S.perm.p, accumulate ? 1 : 0, dphi);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

template <int M, int T, int MAXP>
fp_status launch_grad(fp_ctx* c, hipStream_t st, const Prepared& pp, const fpk::GradArgs& a, const IfcState& S,
                      const double* dldg, double* dphi, bool accumulate) {
    auto kern = fpk::k_grad<M, T, MAXP>;
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, 0));
    if (occ < 1) occ = 1;
    const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * occ, pp.n_units));
    const int ncomp = M == 3 ? 27 : 81;
    const int64_t per = (int64_t)S.n_terms * ncomp;
    HIP_TRY(c, c->gpart.ensure((size_t)(nblk * per)));
    hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(nblk * per)), dim3(256), 0, st, c->gpart.p, nblk * per, 0.0);
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), 0, st, c->omega.p, c->evec.p, c->occ.p,
                       c->roots.p, c->phit.p, S.tmeta.p, S.tc.p, S.groups.p, S.pairs.p, S.scale.p, c->rows.p,
                       c->units.p, dldg, c->gpart.p, c->flag, a);
    HIP_TRY(c, hipGetLastError());
    return reduce_partials(c, st, nblk, S, ncomp, accumulate, dphi);
}

// Second pass of the order-4 adjoint, tuple form: one partial dPhi per wave of
// the largest grid the kernel can keep resident, zeroed once per call
// (grad4t_begin), added to by every row range (launch_grad4t, whose grid never
// exceeds that one) and summed once at the end (reduce_partials).
int64_t grad4t_waves(fp_ctx* c, int* occ_out) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fpk::k_grad4t, fpk::kBlock,
                                                     (size_t)c->L * sizeof(double2)) != hipSuccess || occ < 1)
        occ = 1;
    *occ_out = occ;
    return (int64_t)c->n_cu * occ * fpk::kWavesPerBlock;
}

fp_status grad4t_begin(fp_ctx* c, hipStream_t st, const IfcState& S, int64_t* n_waves) {
    int occ = 0;
    *n_waves = grad4t_waves(c, &occ);
    const int64_t n = *n_waves * (int64_t)S.n_terms * 81;
    HIP_TRY(c, c->gpart.ensure((size_t)n));
    hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n)), dim3(256), 0, st, c->gpart.p, n, 0.0);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

fp_status launch_grad4t(fp_ctx* c, hipStream_t st, const Prepared& pp, const fpk::GradArgs& a, const IfcState& S) {
    auto kern = fpk::k_grad4t;
    const size_t shm = (size_t)c->L * sizeof(double2);  // the root table
    int occ = 0;
    const int64_t cap = grad4t_waves(c, &occ) / fpk::kWavesPerBlock;
    const int64_t n_items = pp.n_units * (int64_t)S.n_groups;
    const int64_t want = (n_items + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    const int64_t nblk = std::max<int64_t>(1, std::min<int64_t>(cap, want));
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), shm, st, c->evec.p, c->roots.p, S.tmeta.p, S.tc.p,
                       S.groups.p, S.scale.p, c->rows.p, c->units.p, c->hbuf.p, c->hdec.p, c->gpart.p, c->flag, a);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

template <int M, int T>
fp_status launch_grad_p(fp_ctx* c, hipStream_t st, const Prepared& pp, const fpk::GradArgs& a, const IfcState& S,
                        const double* dldg, double* dphi, bool accumulate) {
    if (S.n_pairs <= 16) return launch_grad<M, T, 4>(c, st, pp, a, S, dldg, dphi, accumulate);
    return launch_grad<M, T, 8>(c, st, pp, a, S, dldg, dphi, accumulate);
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

namespace {

// Buffers of one ctx swapped for views into the fixed workspace for the length
// of one call, and restored when the call returns on any path.
struct WorkspaceLoan {
    fp_ctx* c;
    DevBuf<double> occ, partial;
    DevBuf<fpk::RowInfo> rows;
    DevBuf<int64_t> row_units, unit_off;
    DevBuf<fpk::UnitDesc> units;
    DevBuf<double2> phit;
    DevBuf<uint4> fsp;
    bool profile;
    template <class T>
    static void lend(DevBuf<T>& b, DevBuf<T>& keep, unsigned char* base, size_t off, size_t n) {
        keep = b;
        b.p = reinterpret_cast<T*>(base + off);
        b.n = n;
        b.borrowed = true;
    }
    ~WorkspaceLoan() {
        c->occ = occ; c->partial = partial; c->rows = rows; c->row_units = row_units;
        c->unit_off = unit_off; c->units = units; c->phit = phit; c->fsp = fsp;
        c->profile = profile;
    }
};

}  // namespace

extern "C" fp_status fp_rates4_noalloc(fp_ctx* c, const fp_plist* lists, int32_t n_lists, int32_t n_T,
                                       const double* T_K, double sigma, int32_t precision, double* gamma_out,
                                       double* wp_out, void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!c->scratch) return fail(c, FP_ERR_HIP, "the no-allocation workspace has no device address");
    fp_status cs = check_common(c, n_lists, lists, n_T, T_K, sigma);
    if (cs != FP_OK) return cs;
    const IfcState& S = c->ifc[1];
    if (S.order != 4) return fail(c, FP_ERR_STATE, "force constants of order 4 not loaded");
    const bool mixed = (precision & ~FP_ACCUMULATE) == FP_MIXED;
    // the sizes run_rates will ask for, laid out in the workspace (256-byte aligned)
    const int64_t unit = (int64_t)fpk::kWave * unit_ppl(c, 4, mixed);
    int64_t total_rows = 0, n_units = 0;
    for (int l = 0; l < n_lists; ++l) {
        total_rows += lists[l].n_rows;
        n_units += (lists[l].n_rec + unit - 1) / unit + lists[l].n_rows;
    }
    const int64_t nu = std::max<int64_t>(n_units, 1);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return at;
    };
    const size_t o_occ = take((size_t)n_T * c->n_modes * 8);
    const size_t o_rows = take((size_t)total_rows * sizeof(fpk::RowInfo));
    const size_t o_ru = take((size_t)(total_rows + 1) * 8);
    const size_t o_uo = take((size_t)(total_rows + 1) * 8);
    const size_t o_units = take((size_t)nu * sizeof(fpk::UnitDesc));
    const size_t o_phit = take((size_t)total_rows * S.n_keys * 27 * sizeof(double2));
    const size_t o_part = take((size_t)nu * 2 * n_T * 8);
    const size_t n_fsp = mixed ? (size_t)total_rows * S.n_kblk * 4 * fpk::kWave * 3 : 1;
    const size_t o_fsp = take(n_fsp * sizeof(uint4));
    if (off > kNoAllocBytes)
        return fail(c, FP_ERR_UNSUPPORTED, "fp_rates4_noalloc needs %zu bytes of workspace, the maximum is %zu",
                    off, kNoAllocBytes);
    HIP_TRY(c, hipSetDevice(c->device));
    unsigned char* base = static_cast<unsigned char*>(c->scratch);
    WorkspaceLoan loan{c, {}, {}, {}, {}, {}, {}, {}, {}, c->profile};
    WorkspaceLoan::lend(c->occ, loan.occ, base, o_occ, (size_t)n_T * c->n_modes);
    WorkspaceLoan::lend(c->rows, loan.rows, base, o_rows, (size_t)std::max<int64_t>(total_rows, 1));
    WorkspaceLoan::lend(c->row_units, loan.row_units, base, o_ru, (size_t)total_rows + 1);
    WorkspaceLoan::lend(c->unit_off, loan.unit_off, base, o_uo, (size_t)total_rows + 1);
    WorkspaceLoan::lend(c->units, loan.units, base, o_units, (size_t)nu);
    WorkspaceLoan::lend(c->phit, loan.phit, base, o_phit, (size_t)std::max<int64_t>(total_rows * S.n_keys * 27, 1));
    WorkspaceLoan::lend(c->partial, loan.partial, base, o_part, (size_t)nu * 2 * n_T);
    WorkspaceLoan::lend(c->fsp, loan.fsp, base, o_fsp, n_fsp);
    c->profile = false;  // kernel timing would create events
    return run_rates(c, 4, lists, n_lists, n_T, T_K, sigma, precision, gamma_out, wp_out, stream);
}

namespace {

// Form of the fused kernel: FP64 0 (B-keys) or 2 (first partner folded), the
// fused_form knob; mixed 1 (split bf16 build) or 3 (the folded form in FP32).
// The folded forms keep the unit's table in LDS (n_pkeys x 54 complex), so
// tables beyond 48 KB (FP64) take the unfolded form.
int fused_form_of(const fp_ctx* c, const IfcState& S, bool mixed) {
    const bool fits = (size_t)S.n_pkeys * fpk::kXM * 16 <= (48u << 10);
    if (mixed) return c->fused_form == 2 && fits ? 3 : 1;
    return c->fused_form == 2 && fits ? 2 : 0;
}

template <int T>
fp_status launch_fused(fp_ctx* c, hipStream_t st, const fpk::RatesArgs& a, const fpk::FusedArgs& f,
                       const IfcState& S, bool mixed) {
    const int form = fused_form_of(c, S, mixed);
    auto kern = form == 1   ? (f.vel ? fpk::k_fused4<T, true, 1> : fpk::k_fused4<T, false, 1>)
                : form == 0 ? (f.vel ? fpk::k_fused4<T, true, 0> : fpk::k_fused4<T, false, 0>)
                : form == 2 ? (f.vel ? fpk::k_fused4<T, true, 2> : fpk::k_fused4<T, false, 2>)
                            : (f.vel ? fpk::k_fused4<T, true, 3> : fpk::k_fused4<T, false, 3>);
    // the FP64 forms also stage the B-key or pkey table when the key table is staged
    const bool xf = form >= 2;
    const int32_t n_tab = xf ? S.n_pkeys : S.n_bkeys;
    const bool staged = S.n_keys <= fpk::kStageTerms && n_tab <= fpk::kStageTerms;
    size_t shm = fpk::tb_dyn_lds(c->L, S.n_keys) + (form != 1 && staged ? (size_t)n_tab * 8 * sizeof(int32_t) : 0);
    if (xf)  // the folded table (complex FP64, or FP32 in form 3), 16-byte aligned after the staged tables
        shm = (size_t)c->L * sizeof(double2) + (staged ? ((size_t)(S.n_keys + n_tab) * 8 + 3) / 4 * 16 : 0) +
              (size_t)S.n_pkeys * fpk::kXM * (form == 3 ? sizeof(float2) : sizeof(double2));
    int occ = 0;
    HIP_TRY(c, hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, fpk::kBlock, shm));
    if (occ < 1) occ = 1;
    const int bpc = c->blocks_per_cu > 0 ? std::min(c->blocks_per_cu, occ) : occ;
    // a unit per wave (form 2: per block)
    const int64_t want = xf ? f.n_units : (f.n_units + fpk::kWavesPerBlock - 1) / fpk::kWavesPerBlock;
    int64_t nblk = std::min<int64_t>((int64_t)c->n_cu * bpc, want);
    nblk = std::max<int64_t>(fpk::kXcd, (nblk + fpk::kXcd - 1) / fpk::kXcd * fpk::kXcd);
    // one folded table per wave (FP64 forms)
    fpk::FusedTabs ft;
    ft.btab = S.btab.p;
    ft.fgroups = S.fgroups.p;
    ft.ptab = S.ptab.p;
    ft.plist = S.plist.p;
    ft.pgroups = S.pgroups.p;
    ft.n_bkeys = S.n_bkeys;
    ft.n_pkeys = S.n_pkeys;
    ft.n_pgroups = S.n_pgroups;
    ft.n_fold_ks = xf ? S.n_pks : S.n_fks;
    const int64_t nfold = form != 0 ? 1 : nblk * fpk::kWavesPerBlock * (int64_t)ft.n_fold_ks * 2 * fpk::kWave;
    HIP_TRY(c, c->fold.ensure((size_t)nfold));
    ft.fold = c->fold.p;
    ft.occt = nullptr;
    if (xf) {  // occupations transposed so that one record's temperatures load together
        const int mt = (T + 1) & ~1;
        const int64_t nocc = c->n_modes * mt;
        HIP_TRY(c, c->occt.ensure((size_t)nocc));
        hipLaunchKernelGGL(fpk::k_occ_t, dim3(grid_for(nocc)), dim3(256), 0, st, c->occ.p, c->n_modes, a.n_T, mt,
                           c->occt.p);
        ft.occt = c->occt.p;
    }
    fpk::RatesArgs af = a;
    if (form == 0) af.n_groups = S.n_fgroups;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(fpk::kBlock), shm, st, c->omega.p, c->evec.p, c->occ.p,
                       c->roots.p, c->phit.p, S.tmeta.p, S.groups.p, c->rows.p, c->partial.p, c->unit_kept.p,
                       c->unit_tup.p, c->flag, af, f, c->evec32.p, c->fsp.p, S.n_kblk, ft);
    HIP_TRY(c, hipGetLastError());
    return FP_OK;
}

}  // namespace

extern "C" fp_status fp_rates4_fused(fp_ctx* c, int64_t n_rows, const int32_t* row_mode, int32_t type_mask,
                                     int32_t n_T, const double* T_K, double sigma, double nsigma, int32_t precision,
                                     double* gamma_out, double* wp_out, int64_t* n_kept, void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes has not been called");
    IfcState& S = c->ifc[1];
    if (S.order != 4) return fail(c, FP_ERR_STATE, "force constants of order 4 not loaded");
    if (c->nb != fpk::kFusedNb) return fail(c, FP_ERR_UNSUPPORTED, "the fused path is built for nb = 6 (two atoms)");
    if (n_rows < 0 || (n_rows > 0 && !row_mode)) return fail(c, FP_ERR_ARG, "bad row list");
    if (type_mask < 1 || type_mask > 7) return fail(c, FP_ERR_ARG, "type_mask must be in [1, 7]");
    if (n_T < 1 || n_T > FP_MAX_T || !T_K) return fail(c, FP_ERR_ARG, "n_T must be in [1, %d]", FP_MAX_T);
    for (int i = 0; i < n_T; ++i)
        if (!(T_K[i] > 0.0)) return fail(c, FP_ERR_ARG, "temperatures must be positive");
    if (!(sigma > 0.0) || !(nsigma > 0.0)) return fail(c, FP_ERR_ARG, "sigma and nsigma must be positive");
    const bool accumulate = (precision & FP_ACCUMULATE) != 0;
    const int32_t prec = precision & ~FP_ACCUMULATE;
    if (prec != FP_FP64 && prec != FP_MIXED) return fail(c, FP_ERR_ARG, "unknown precision %d", prec);
    const bool mixed = prec == FP_MIXED;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nm = c->n_modes;
    if (gamma_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, gamma_out, n_T * nm, 0.0);
    if (wp_out && !accumulate)
        hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, wp_out, n_T * nm, 0.0);
    HIP_TRY(c, c->fused_cnt.ensure(2));
    if (n_rows == 0) {
        if (n_kept) hipLaunchKernelGGL(fpk::k_sum_i64, dim3(1), dim3(fpk::kBlock), 0, st, (const int64_t*)nullptr,
                                       (int64_t)0, n_kept);
        for (int i = 0; i < 2; ++i)
            hipLaunchKernelGGL(fpk::k_sum_i64, dim3(1), dim3(fpk::kBlock), 0, st, (const int64_t*)nullptr,
                               (int64_t)0, c->fused_cnt.p + i);
        HIP_TRY(c, hipGetLastError());
        c->fused_done = true;
        return FP_OK;
    }
    fpk::FusedArgs f;
    memset(&f, 0, sizeof f);
    for (int t = 0; t < 3; ++t)
        if (type_mask & (1 << t)) f.types[f.n_types++] = FP_4PP + t;
    f.n_rows = n_rows;
    f.n_units = (int64_t)f.n_types * n_rows * c->nq;
    f.floor_ = c->floor_;
    // extreme frequencies of the mesh for the kernel's unit bound (active modes for the minimum)
    f.wmin = std::numeric_limits<double>::infinity();
    f.wmax = 0.0;
    for (double w : c->h_omega) {
        if (w >= c->floor_) f.wmin = std::min(f.wmin, w);
        f.wmax = std::max(f.wmax, w);
    }
    f.cut = nsigma * sigma;
    if (c->adaptive) {
        // the enumerator's rule; cut_max bounds nsigma * sigma_p over every process
        f.vel = c->vel.p;
        f.proj = c->proj.p;
        f.proj_max = c->proj_max.p;
        for (int i = 0; i < 9; ++i) f.recip[i] = c->bro.recip[i];
        f.factor = c->bro.factor;
        f.sigma = sigma;
        f.nsigma = nsigma;
        double pmax[3] = {0.0, 0.0, 0.0};
        for (int64_t g = 0; g < nm; ++g)
            for (int d = 0; d < 3; ++d) {
                const double* v = c->h_vel.data() + g * 3;
                const double p = std::fabs(v[0] * f.recip[d * 3] + v[1] * f.recip[d * 3 + 1] + v[2] * f.recip[d * 3 + 2]) /
                                 (double)c->mesh[d];
                pmax[d] = std::max(pmax[d], p);
            }
        double babs = 0.0;  // max over modes and directions of sum_k |v_k b_dk| / N_d
        for (int64_t g = 0; g < nm; ++g)
            for (int d = 0; d < 3; ++d) {
                const double* v = c->h_vel.data() + g * 3;
                const double p = (std::fabs(v[0] * f.recip[d * 3]) + std::fabs(v[1] * f.recip[d * 3 + 1]) +
                                  std::fabs(v[2] * f.recip[d * 3 + 2])) / (double)c->mesh[d];
                babs = std::max(babs, p);
            }
        f.perr = 3e-12 * babs;
        double b2 = 0.0;
        for (int d = 0; d < 3; ++d) b2 += 4.0 * pmax[d] * pmax[d];
        const double smax = std::max(f.factor * std::sqrt(3.0 * b2 / 9.0), sigma);
        f.cut_max = nsigma * smax * (1.0 + 1e-9);
    }
    const int64_t n_frows = (int64_t)f.n_types * n_rows;
    HIP_TRY(c, c->occ.ensure((size_t)n_T * nm));
    HIP_TRY(c, c->rows.ensure((size_t)n_frows));
    HIP_TRY(c, c->unit_off.ensure((size_t)n_frows + 1));
    HIP_TRY(c, c->phit.ensure((size_t)n_frows * S.n_keys * 27));
    HIP_TRY(c, c->partial.ensure((size_t)f.n_units * 2 * n_T));
    HIP_TRY(c, c->unit_kept.ensure((size_t)f.n_units));
    HIP_TRY(c, c->unit_tup.ensure((size_t)f.n_units));
    fpk::Temps tx;
    for (int i = 0; i < 8; ++i) tx.x[i] = i < n_T ? kHbar / (kBoltz * T_K[i]) : 0.0;
    hipLaunchKernelGGL(fpk::k_occ, dim3(grid_for(n_T * nm)), dim3(256), 0, st, c->omega.p, nm, n_T, tx, c->floor_,
                       c->occ.p);
    hipLaunchKernelGGL(fpk::k_fused_rows, dim3(grid_for(n_frows + 1)), dim3(256), 0, st, row_mode, f, (int64_t)c->nq,
                       nm, c->rows.p, c->unit_off.p, c->flag);
    const fpk::ModeGeom geo = geometry(c);
    hipLaunchKernelGGL(fpk::k_precontract<4>, dim3(grid_for(n_frows * S.n_keys * 27)), dim3(256), 0, st, c->rows.p,
                       n_frows, c->evec.p, c->roots.p, geo, S.phi_s.p, S.tmeta.p, S.tc.p, S.n_keys, c->phit.p);
    if (fused_form_of(c, S, mixed) == 1) {  // the split bf16 force constants of form 1
        const int64_t nf = n_frows * S.n_kblk * 4 * fpk::kWave;
        HIP_TRY(c, c->fsp.ensure((size_t)std::max<int64_t>(nf * 3, 1)));
        hipLaunchKernelGGL(fpk::k_split_phit, dim3(grid_for(nf)), dim3(256), 0, st, n_frows, c->phit.p, S.groups.p,
                           S.kblk.p, S.n_kblk, (int32_t)S.n_keys, c->fsp.p);
    }
    HIP_TRY(c, hipGetLastError());
    fpk::RatesArgs a;
    memset(&a, 0, sizeof a);
    a.n_units = f.n_units;
    a.n_modes = nm;
    a.n_keys = (int32_t)S.n_keys;
    a.n_groups = S.n_groups;
    a.n_T = n_T;
    a.ppl = fpk::kBR;
    a.geo = geo;
    a.br = make_broad(c, sigma);
    const int tsel = n_T == 1 ? 1 : (n_T <= 4 ? 4 : 8);
    hipEvent_t ev0, ev1;
    fp_status ts = timer_start(c, st, &ev0, &ev1);
    if (ts != FP_OK) return ts;
    fp_status ls = tsel == 1 ? launch_fused<1>(c, st, a, f, S, mixed)
                             : (tsel == 4 ? launch_fused<4>(c, st, a, f, S, mixed) : launch_fused<8>(c, st, a, f, S, mixed));
    if (ls != FP_OK) return ls;
    ts = timer_stop(c, st, 34, ev0, ev1);
    if (ts != FP_OK) return ts;
    const double pref = rate_prefactor(c, 4);
    const double wpref = 1.0 / ((double)c->nq * (double)c->nq);
    // kept processes and tuples of the call: per-block parts, then one block over the parts
    constexpr int kParts = 256;
    HIP_TRY(c, c->sum_parts.ensure(2 * kParts));
    hipLaunchKernelGGL(fpk::k_sum_i64_parts, dim3(kParts), dim3(fpk::kBlock), 0, st, c->unit_kept.p, f.n_units,
                       c->sum_parts.p);
    hipLaunchKernelGGL(fpk::k_sum_i64_parts, dim3(kParts), dim3(fpk::kBlock), 0, st, c->unit_tup.p, f.n_units,
                       c->sum_parts.p + kParts);
    if (n_kept)
        hipLaunchKernelGGL(fpk::k_sum_i64, dim3(1), dim3(fpk::kBlock), 0, st, c->sum_parts.p, (int64_t)kParts, n_kept);
    hipLaunchKernelGGL(fpk::k_sum_i64, dim3(1), dim3(fpk::kBlock), 0, st, c->sum_parts.p, (int64_t)kParts,
                       c->fused_cnt.p);
    hipLaunchKernelGGL(fpk::k_sum_i64, dim3(1), dim3(fpk::kBlock), 0, st, c->sum_parts.p + kParts, (int64_t)kParts,
                       c->fused_cnt.p + 1);
    c->fused_done = true;
    // one finalize launch per type: rows of one mode in different types add into the same outputs
    for (int ti = 0; ti < f.n_types; ++ti)
        hipLaunchKernelGGL(fpk::k_finalize, dim3((unsigned)n_rows), dim3(fpk::kBlock), 0, st, c->partial.p,
                           c->unit_off.p, c->rows.p, (int64_t)ti * n_rows, n_T, pref, wpref, gamma_out, wp_out, nm);
    HIP_TRY(c, hipGetLastError());
    if (c->validate) return fp_check(c, stream);
    return FP_OK;
}

extern "C" fp_status fp_peak_probe(fp_ctx* c, int32_t kind, int32_t reps, double* achieved, void* stream) {
    if (!c || !achieved) return FP_ERR_ARG;
    if (kind < 0 || kind > 4) return fail(c, FP_ERR_ARG, "probe kind must be in [0, 4]");
    if (reps < 1 || reps > 100) return fail(c, FP_ERR_ARG, "reps must be in [1, 100]");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    // FLOP (or bytes) of one launch and the launch itself
    const int64_t blocks = (int64_t)c->n_cu * (kind == 0 ? 8 : 4);
    const int iters = kind == 0 ? 16384 : (kind == 3 ? 16384 : 4096);
    const int64_t n_copy = int64_t(1) << 26;  // 16-byte elements: 1 GiB each way
    DevBuf<uint4> src, dst;
    if (kind == 4) {
        HIP_TRY(c, src.ensure((size_t)n_copy));
        HIP_TRY(c, dst.ensure((size_t)n_copy));
    } else {
        HIP_TRY(c, c->probe_out.ensure((size_t)(blocks * fpk::kBlock)));
    }
    double work = 0.0;
    auto launch = [&]() {
        switch (kind) {
            case 0:
                hipLaunchKernelGGL(fpk::k_probe_fma64, dim3((unsigned)blocks), dim3(fpk::kBlock), 0, st, c->probe_out.p,
                                   iters);
                work = 2.0 * fpk::kProbeChains * (double)iters * (double)(blocks * fpk::kBlock);
                break;
            case 1:
            case 2:
            case 3: {
                auto k = kind == 1 ? fpk::k_probe_mfma<0> : (kind == 2 ? fpk::k_probe_mfma<1> : fpk::k_probe_mfma<2>);
                hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(fpk::kBlock), 0, st, c->probe_out.p, iters);
                const double per = kind == 3 ? 16.0 * 16 * 32 * 2 : 16.0 * 16 * 4 * 2;
                work = per * fpk::kProbeAcc * (double)iters * (double)(blocks * fpk::kWavesPerBlock);
                break;
            }
            default:
                hipLaunchKernelGGL(fpk::k_probe_copy, dim3((unsigned)(c->n_cu * 8)), dim3(fpk::kBlock), 0, st, src.p,
                                   dst.p, n_copy);
                work = 2.0 * (double)n_copy * sizeof(uint4);
        }
    };
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, FP_ERR_HIP, "hipEventCreate failed");
    }
    launch();  // untimed
    double best = 0.0;
    hipError_t err = hipGetLastError();
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        err = hipEventRecord(e0, st);
        if (err == hipSuccess) launch();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err == hipSuccess && ms > 0.0f) best = std::max(best, work / (ms * 1e-3));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    src.release();
    dst.release();
    if (err != hipSuccess) return fail(c, FP_ERR_HIP, "peak probe: %s", hipGetErrorString(err));
    *achieved = kind == 4 ? best / 1e9 : best / 1e12;  // GB/s or TFLOP/s
    return FP_OK;
}

extern "C" fp_status fp_fused_counts(fp_ctx* c, int64_t out[2], void* stream) {
    if (!c) return FP_ERR_ARG;
    if (!out) return fail(c, FP_ERR_ARG, "out is NULL");
    if (!c->fused_done) return fail(c, FP_ERR_STATE, "no fp_rates4_fused call on this context");
    HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipMemcpyAsync(out, c->fused_cnt.p, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    return FP_OK;
}

extern "C" fp_status fp_autotune(fp_ctx* c, int32_t order, const fp_plist* lists, int32_t n_lists, int32_t n_T,
                                 const double* T_K, double sigma, int32_t precision, int32_t reps,
                                 fp_tune_entry* report, int32_t n_report, int32_t* n_written, void* stream) {
    if (!c || (order != 3 && order != 4) || reps < 1 || reps > 100 || (n_report > 0 && !report) || n_report < 0)
        return FP_ERR_ARG;
    if (!c->modes) return fail(c, FP_ERR_STATE, "fp_load_modes has not been called");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t nm = c->n_modes;
    if (n_T < 1 || n_T > FP_MAX_T) return fail(c, FP_ERR_ARG, "n_T must be in [1, %d]", FP_MAX_T);
    HIP_TRY(c, c->tune_out.ensure((size_t)n_T * nm));
    // candidates: (variant, records per lane, resident blocks per CU)
    struct Cand { int32_t v, ppl, bpc; };
    std::vector<Cand> cands;
    const bool mixed4 = order == 4 && (precision & ~FP_ACCUMULATE) == FP_MIXED;
    if (order == 3) {
        for (int32_t ppl : {1, 2, 4})
            for (int32_t bpc : {0, 1}) cands.push_back({c->variant, ppl, bpc});
    } else if (mixed4) {
        for (int32_t bpc : {0, 1}) cands.push_back({c->variant, 2, bpc});
    } else {
        for (int32_t v = 0; v < 8; ++v) {
            const std::vector<int32_t> ppls = v >= 4 ? std::vector<int32_t>{batched_br(v)}
                                                     : (kVariants[v].np == 1 ? std::vector<int32_t>{1, 2, 4}
                                                                             : std::vector<int32_t>{2, 4});
            for (int32_t ppl : ppls)
                for (int32_t bpc : {0, 1}) cands.push_back({v, ppl, bpc});
        }
    }
    const int32_t keep_v = c->variant, keep_ppl = c->ppl, keep_bpc = c->blocks_per_cu;
    const bool keep_prof = c->profile;
    c->profile = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    double best = 1e300;
    Cand pick = {keep_v, keep_ppl, keep_bpc};
    int32_t written = 0;
    fp_status bad = FP_OK;
    for (const Cand& k : cands) {
        c->variant = k.v;
        c->ppl = k.ppl;
        c->blocks_per_cu = k.bpc;
        const int32_t prec = precision & ~FP_ACCUMULATE;
        // one untimed launch, then `reps` timed ones
        bad = run_rates(c, order, lists, n_lists, n_T, T_K, sigma, prec, c->tune_out.p, nullptr, stream);
        if (bad != FP_OK) break;
        if (hipEventRecord(e0, st) != hipSuccess) { bad = fail(c, FP_ERR_HIP, "event record failed"); break; }
        for (int r = 0; r < reps && bad == FP_OK; ++r)
            bad = run_rates(c, order, lists, n_lists, n_T, T_K, sigma, prec, c->tune_out.p, nullptr, stream);
        if (bad != FP_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            bad = fail(c, FP_ERR_HIP, "event timing failed");
            break;
        }
        const double per = ms / reps;
        if (written < n_report) report[written++] = {k.v, k.ppl, k.bpc, 0, per};
        if (per < best) {
            best = per;
            pick = k;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->profile = keep_prof;
    if (n_written) *n_written = written;
    if (bad != FP_OK) {
        c->variant = keep_v;
        c->ppl = keep_ppl;
        c->blocks_per_cu = keep_bpc;
        return bad;
    }
    c->variant = pick.v;
    c->ppl = pick.ppl;
    c->blocks_per_cu = pick.bpc;
    return FP_OK;
}

extern "C" fp_status fp_rates_backward(fp_ctx* c, const fp_plist* lists, int32_t n_lists, int32_t n_T,
                                       const double* T_K, double sigma, int32_t precision, const double* dL_dgamma,
                                       double* dphi3, double* dphi4, void* stream) {
    if (!c) return FP_ERR_ARG;
    fp_status cs = check_common(c, n_lists, lists, n_T, T_K, sigma);
    if (cs != FP_OK) return cs;
    for (int l = 0; l < n_lists; ++l)
        if (lists[l].type == FP_3E) return fail(c, FP_ERR_UNSUPPORTED, "the adjoint takes per-mode lists, not events");
    const bool accumulate = (precision & FP_ACCUMULATE) != 0;
    precision &= ~FP_ACCUMULATE;
    if (precision != FP_FP64 && precision != FP_MIXED) return fail(c, FP_ERR_ARG, "unknown precision %d", precision);
    const bool mixed = precision == FP_MIXED;
    if (!dL_dgamma) return fail(c, FP_ERR_ARG, "dL_dgamma is null");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    for (int m = 3; m <= 4; ++m) {
        double* dphi = m == 3 ? dphi3 : dphi4;
        if (!dphi) continue;
        IfcState& S = c->ifc[m - 3];
        if (S.order != m) return fail(c, FP_ERR_STATE, "force constants of order %d not loaded", m);
        const int ncomp = m == 3 ? 27 : 81;
        std::vector<int> sel;
        int64_t n_rec = 0, n_rows = 0;
        for (int l = 0; l < n_lists; ++l)
            if (ORDER_OF(lists[l].type) == m) {
                sel.push_back(l);
                n_rec += lists[l].n_rec;
                n_rows += lists[l].n_rows;
            }
        if (n_rows == 0) {
            if (!accumulate)
                hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(S.n_terms * ncomp)), dim3(256), 0, st, dphi,
                                   S.n_terms * ncomp, 0.0);
            HIP_TRY(c, hipGetLastError());
            continue;
        }
        const int tsel = n_T == 1 ? 1 : (n_T <= 4 ? 4 : 8);
        hipEvent_t ev0, ev1;
        fp_status ts = timer_start(c, st, &ev0, &ev1);
        if (ts != FP_OK) return ts;
        Prepared pp;
        fp_status ps;
        fpk::GradArgs a;
        memset(&a, 0, sizeof a);
        a.n_modes = c->n_modes;
        a.n_terms = (int32_t)S.n_terms;
        a.n_keys = (int32_t)S.n_keys;
        a.n_groups = S.n_groups;
        a.n_pairs = S.n_pairs;
        a.n_T = n_T;
        a.br = make_broad(c, sigma);
        a.pref = rate_prefactor(c, m);
        if (m == 4 && n_rec > 0) {
            // Row ranges of at most grad_records records (a longer row alone) are
            // taken one after another, so the h buffer of the first pass holds one
            // range, not the whole call: pass 1 writes h_p = c_p conj(V_p) per record
            // of the range (tuple-batched, units of 128 records, FP64 or mixed), pass
            // 2 turns it into dL/dPhi, added over the ranges in order.
            std::vector<std::vector<int64_t>> offs(sel.size());
            for (size_t k = 0; k < sel.size(); ++k) {
                const fp_plist& P = lists[sel[k]];
                offs[k].resize((size_t)P.n_rows + 1);
                HIP_TRY(c, hipMemcpyAsync(offs[k].data(), P.row_off, offs[k].size() * 8, hipMemcpyDeviceToHost, st));
            }
            HIP_TRY(c, hipStreamSynchronize(st));
            struct Piece { size_t k; int64_t r0, r1; };
            std::vector<std::vector<Piece>> ranges(1);
            int64_t cur = 0;
            for (size_t k = 0; k < sel.size(); ++k)
                for (int64_t r = 0; r < lists[sel[k]].n_rows; ++r) {
                    const int64_t nr = offs[k][(size_t)r + 1] - offs[k][(size_t)r];
                    if (nr < 0 || offs[k][(size_t)r] < 0 || offs[k][(size_t)r + 1] > lists[sel[k]].n_rec)
                        return fail(c, FP_ERR_ARG, "list %d: bad row offsets", sel[k]);
                    if (cur > 0 && cur + nr > c->grad_records) {
                        ranges.emplace_back();
                        cur = 0;
                    }
                    auto& rg = ranges.back();
                    if (!rg.empty() && rg.back().k == k && rg.back().r1 == r)
                        rg.back().r1 = r + 1;
                    else
                        rg.push_back({k, r, r + 1});
                    cur += nr;
                }
            // the h buffer at the largest range's size up front (no reallocation,
            // hence no device-wide wait, between ranges)
            int64_t max_range = 1;
            for (const auto& rg : ranges) {
                int64_t nr = 0;
                for (const Piece& pc : rg) nr += offs[pc.k][(size_t)pc.r1] - offs[pc.k][(size_t)pc.r0];
                max_range = std::max(max_range, nr);
            }
            HIP_TRY(c, c->hbuf.ensure((size_t)max_range));
            HIP_TRY(c, c->hdec.ensure((size_t)max_range));
            const double pref4 = rate_prefactor(c, m);
            int64_t n_waves = 0;
            ps = grad4t_begin(c, st, S, &n_waves);
            if (ps != FP_OK) return ps;
            for (size_t ri = 0; ri < ranges.size(); ++ri) {
                std::vector<fp_plist> sub;
                std::vector<int64_t> shift;
                std::vector<int> all;
                int64_t n_sub = 0;
                for (const Piece& pc : ranges[ri]) {
                    const fp_plist& P = lists[sel[pc.k]];
                    const int64_t b0 = offs[pc.k][(size_t)pc.r0], b1 = offs[pc.k][(size_t)pc.r1];
                    fp_plist q = P;
                    q.n_rows = pc.r1 - pc.r0;
                    q.n_rec = b1 - b0;
                    q.row_mode = P.row_mode + pc.r0;
                    q.row_off = P.row_off + pc.r0;
                    q.rec = P.rec + b0;
                    all.push_back((int)sub.size());
                    sub.push_back(q);
                    shift.push_back(b0);
                    n_sub += b1 - b0;
                }
                ps = prepare(c, m, sub.data(), all, n_T, T_K, fpk::kBR * fpk::kWave, st, &pp, &shift);
                if (ps != FP_OK) return ps;
                HIP_TRY(c, c->hbuf.ensure((size_t)std::max<int64_t>(n_sub, 1)));
                HIP_TRY(c, c->hdec.ensure((size_t)std::max<int64_t>(n_sub, 1)));
                fpk::RatesArgs ra;
                memset(&ra, 0, sizeof ra);
                ra.n_units = pp.n_units;
                ra.n_modes = c->n_modes;
                ra.n_keys = (int32_t)S.n_keys;
                ra.n_groups = S.n_groups;
                ra.n_T = n_T;
                ra.ppl = fpk::kBR;
                ra.geo = pp.geo;
                ra.br = make_broad(c, sigma);
                if (mixed) {
                    const int64_t nf = pp.total_rows * S.n_kblk * 4 * fpk::kWave;
                    HIP_TRY(c, c->fsp.ensure((size_t)std::max<int64_t>(nf * 3, 1)));
                    hipLaunchKernelGGL(fpk::k_split_phit, dim3(grid_for(nf)), dim3(256), 0, st, pp.total_rows,
                                       c->phit.p, S.groups.p, S.kblk.p, S.n_kblk, (int32_t)S.n_keys, c->fsp.p);
                    ps = tsel == 1 ? launch_mixed_h<1>(c, st, pp.n_units, ra, S, dL_dgamma, pref4)
                                   : (tsel == 4 ? launch_mixed_h<4>(c, st, pp.n_units, ra, S, dL_dgamma, pref4)
                                                : launch_mixed_h<8>(c, st, pp.n_units, ra, S, dL_dgamma, pref4));
                } else {
                    ps = tsel == 1 ? launch_batched_h<1>(c, st, pp.n_units, ra, S, dL_dgamma, pref4)
                                   : (tsel == 4 ? launch_batched_h<4>(c, st, pp.n_units, ra, S, dL_dgamma, pref4)
                                                : launch_batched_h<8>(c, st, pp.n_units, ra, S, dL_dgamma, pref4));
                }
                if (ps != FP_OK) return ps;
                ps = prepare(c, m, sub.data(), all, n_T, T_K, c->grad_chunk, st, &pp, &shift);
                if (ps != FP_OK) return ps;
                a.n_units = pp.n_units;
                a.geo = pp.geo;
                fp_status ls = launch_grad4t(c, st, pp, a, S);
                if (ls != FP_OK) return ls;
            }
            ps = reduce_partials(c, st, n_waves, S, 81, accumulate, dphi);
            if (ps != FP_OK) return ps;
        } else {
            ps = prepare(c, m, lists, sel, n_T, T_K, c->grad_chunk, st, &pp);
            if (ps != FP_OK) return ps;
            a.n_units = pp.n_units;
            a.geo = pp.geo;
            fp_status ls;
            if (m == 3)
                ls = tsel == 1 ? launch_grad_p<3, 1>(c, st, pp, a, S, dL_dgamma, dphi, accumulate)
                               : (tsel == 4 ? launch_grad_p<3, 4>(c, st, pp, a, S, dL_dgamma, dphi, accumulate)
                                            : launch_grad_p<3, 8>(c, st, pp, a, S, dL_dgamma, dphi, accumulate));
            else
            {
                int64_t n_waves = 0;
                ls = grad4t_begin(c, st, S, &n_waves);
                if (ls == FP_OK) ls = launch_grad4t(c, st, pp, a, S);
                if (ls == FP_OK) ls = reduce_partials(c, st, n_waves, S, 81, accumulate, dphi);
            }
            if (ls != FP_OK) return ls;
        }
        ts = timer_stop(c, st, 10 + m, ev0, ev1);
        if (ts != FP_OK) return ts;
    }
    if (c->validate) return fp_check(c, stream);
    return FP_OK;
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
    if (!c || !total_ms || !launches || (order != 3 && order != 4 && order != 13 && order != 14 && order != 24 &&
                                               order != 34))
        return FP_ERR_ARG;
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

// ------------------------------------------------------- streaming executor
//
// Mode-wise fallback generalised to chunks (Appendix, the mode-wise variant of
// Algorithm 4; Results, memory limits of the all-modes strategy): the host
// enumerator counts every selected (type, row), the concatenated record
// sequence is cut into chunks of at most chunk_records, and each chunk is
// enumerated into a pinned staging slot, copied to the device and evaluated by
// the ordinary rate launches with FP_ACCUMULATE.  Two slots alternate, so the
// host fills chunk k+1 while the GPU copies and evaluates chunk k.

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

struct EnumSet {
    fpenum::Handle* h[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    ~EnumSet() {
        for (auto* p : h) fpenum::close(p);
    }
};

}  // namespace

extern "C" fp_status fp_rates_streamed(fp_ctx* c, int32_t type_mask, int64_t n_rows, const int32_t* row_mode,
                                       int32_t n_T, const double* T_K, double sigma, double nsigma,
                                       int32_t precision, int64_t chunk_records, int32_t n_threads,
                                       double* gamma_out, double* wp_out, fp_stream_stats* stats, void* stream) {
    if (!c) return FP_ERR_ARG;
    const Clock::time_point t_call = Clock::now();
    fp_status cs = check_common(c, 0, nullptr, n_T, T_K, sigma);
    if (cs != FP_OK) return cs;
    if (type_mask < 1 || type_mask > 31) return fail(c, FP_ERR_ARG, "type_mask must be in [1, 31]");
    if (!(nsigma > 0.0) || !std::isfinite(nsigma)) return fail(c, FP_ERR_ARG, "nsigma must be > 0");
    if (chunk_records < 1 || chunk_records > (int64_t(1) << 32))
        return fail(c, FP_ERR_ARG, "chunk_records must be in [1, 2^32]");
    const bool accumulate = (precision & FP_ACCUMULATE) != 0;
    const int32_t prec = precision & ~FP_ACCUMULATE;
    if (prec != FP_FP64 && prec != FP_MIXED) return fail(c, FP_ERR_ARG, "unknown precision %d", prec);
    if (n_rows < 0 || (n_rows > 0 && !row_mode)) return fail(c, FP_ERR_ARG, "bad row list");
    {
        std::vector<int32_t> sorted(row_mode, row_mode + n_rows);
        std::sort(sorted.begin(), sorted.end());
        for (int64_t r = 0; r < n_rows; ++r) {
            if (sorted[r] < 0 || sorted[r] >= c->n_modes) return fail(c, FP_ERR_ARG, "row mode out of range");
            if (r > 0 && sorted[r] == sorted[r - 1]) return fail(c, FP_ERR_ARG, "row modes must be distinct");
        }
    }
    std::vector<int32_t> ts;  // selected types, ascending
    for (int32_t t = FP_3P; t <= FP_4MM; ++t) {
        if (!(type_mask & (1 << t))) continue;
        const int m = t <= FP_3M ? 3 : 4;
        if (c->ifc[m - 3].order != m) return fail(c, FP_ERR_STATE, "force constants of order %d not loaded", m);
        ts.push_back(t);
    }
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(c, hipSetDevice(c->device));
    // a previous call that stopped on an error may have left copies from the
    // staging slots in flight
    for (StreamSlot& sl : c->slot)
        if (sl.done) HIP_TRY(c, hipEventSynchronize(sl.done));
    const int64_t nm = c->n_modes;
    if (!accumulate) {
        if (gamma_out)
            hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, gamma_out, n_T * nm, 0.0);
        if (wp_out)
            hipLaunchKernelGGL(fpk::k_fill, dim3(grid_for(n_T * nm)), dim3(256), 0, st, wp_out, n_T * nm, 0.0);
        HIP_TRY(c, hipGetLastError());
    }
    EnumSet es;
    for (int32_t t : ts) {
        fp_status s = fpenum::open(&es.h[t], t, c->mesh, c->nb, c->h_omega.data(), c->floor_, sigma, nsigma,
                                   c->adaptive ? c->h_vel.data() : nullptr, c->adaptive ? &c->bro : nullptr);
        if (s != FP_OK) return fail(c, s, "enumerator setup failed for type %d", t);
    }

    // count pass: records of every (type, row), types major
    const int64_t n_seq = (int64_t)ts.size() * n_rows;
    Clock::time_point t0 = Clock::now();
    std::vector<int64_t> goff((size_t)n_seq + 1, 0);
    fpenum::parallel_for(n_seq, n_threads, [&](int64_t i) {
        goff[(size_t)i + 1] = fpenum::count_row(es.h[ts[(size_t)(i / n_rows)]], row_mode[i % n_rows]);
    });
    for (int64_t i = 0; i < n_seq; ++i) goff[(size_t)i + 1] += goff[(size_t)i];
    const double count_ms = ms_since(t0);
    const int64_t total = goff[(size_t)n_seq];
    const int64_t cap = std::min(chunk_records, std::max<int64_t>(total, 1));
    const int64_t n_chunks = (total + cap - 1) / cap;
    const size_t nt = ts.size();

    double fill_ms = 0.0, wait_ms = 0.0;
    int64_t max_chunk = 0;
    struct Seg {
        int64_t seq;        // (type, row) index in the global sequence
        int64_t beg, end;   // record window within the row
        int64_t dst;        // position in the chunk
    };
    std::vector<Seg> segs;
    for (int64_t k = 0; k < n_chunks; ++k) {
        StreamSlot& sl = c->slot[k & 1];
        if (!sl.done) HIP_TRY(c, hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
        if (k >= 2) {
            t0 = Clock::now();
            HIP_TRY(c, hipEventSynchronize(sl.done));
            wait_ms += ms_since(t0);
        }
        HIP_TRY(c, sl.rec.ensure((size_t)cap));
        HIP_TRY(c, sl.off.ensure((size_t)(n_seq + nt)));
        HIP_TRY(c, sl.mode.ensure((size_t)std::max<int64_t>(n_seq, 1)));
        HIP_TRY(c, sl.drec.ensure((size_t)cap));
        HIP_TRY(c, sl.doff.ensure((size_t)(n_seq + nt)));
        HIP_TRY(c, sl.dmode.ensure((size_t)std::max<int64_t>(n_seq, 1)));
        const int64_t lo = k * cap, hi = std::min(total, lo + cap);
        max_chunk = std::max(max_chunk, hi - lo);
        // the (type, row) entries overlapping [lo, hi)
        segs.clear();
        int64_t i = std::upper_bound(goff.begin(), goff.end(), lo) - goff.begin() - 1;
        for (; i < n_seq && goff[(size_t)i] < hi; ++i) {
            const int64_t b = std::max(goff[(size_t)i], lo), e = std::min(goff[(size_t)i + 1], hi);
            if (e > b) segs.push_back({i, b - goff[(size_t)i], e - goff[(size_t)i], b - lo});
        }
        // per-type row tables of this chunk: modes, then offsets into the chunk's records
        int n3 = 0, n4 = 0;
        fp_plist l3[2], l4[3];
        int64_t mpos = 0, opos = 0;
        size_t sj = 0;
        for (size_t ti = 0; ti < nt; ++ti) {
            fp_plist P;
            memset(&P, 0, sizeof P);
            P.type = ts[ti];
            const int64_t m0 = mpos, o0 = opos;
            int64_t first = -1, last = 0;
            for (; sj < segs.size() && segs[sj].seq / n_rows == (int64_t)ti; ++sj) {
                sl.mode.p[mpos++] = row_mode[segs[sj].seq % n_rows];
                sl.off.p[opos++] = segs[sj].dst;
                if (first < 0) first = segs[sj].dst;
                last = segs[sj].dst + (segs[sj].end - segs[sj].beg);
            }
            if (mpos == m0) continue;
            sl.off.p[opos++] = last;
            // offsets relative to the list's first record
            for (int64_t q = o0; q < opos; ++q) sl.off.p[q] -= first;
            P.n_rows = mpos - m0;
            P.n_rec = last - first;
            P.row_mode = sl.dmode.p + m0;
            P.row_off = sl.doff.p + o0;
            P.rec = sl.drec.p + first;
            if (P.type <= FP_3M) l3[n3++] = P;
            else l4[n4++] = P;
        }
        // enumerate the chunk's records on the host threads
        t0 = Clock::now();
        std::vector<int64_t> got(segs.size(), 0);
        fpenum::parallel_for((int64_t)segs.size(), n_threads, [&](int64_t j) {
            const Seg& g = segs[(size_t)j];
            got[(size_t)j] = fpenum::fill_row(es.h[ts[(size_t)(g.seq / n_rows)]], row_mode[g.seq % n_rows], g.beg,
                                              g.end, sl.rec.p + g.dst);
        });
        fill_ms += ms_since(t0);
        for (size_t j = 0; j < segs.size(); ++j)
            if (got[j] != segs[j].end - segs[j].beg)
                return fail(c, FP_ERR_STATE, "enumeration changed between the count and fill passes");
        HIP_TRY(c, hipMemcpyAsync(sl.drec.p, sl.rec.p, (size_t)(hi - lo) * sizeof(uint64_t), hipMemcpyHostToDevice,
                                  st));
        HIP_TRY(c, hipMemcpyAsync(sl.doff.p, sl.off.p, (size_t)opos * sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIP_TRY(c, hipMemcpyAsync(sl.dmode.p, sl.mode.p, (size_t)mpos * sizeof(int32_t), hipMemcpyHostToDevice, st));
        fp_status rs = FP_OK;
        if (n3 > 0) rs = run_rates(c, 3, l3, n3, n_T, T_K, sigma, prec | FP_ACCUMULATE, gamma_out, wp_out, stream);
        if (rs == FP_OK && n4 > 0)
            rs = run_rates(c, 4, l4, n4, n_T, T_K, sigma, prec | FP_ACCUMULATE, gamma_out, wp_out, stream);
        HIP_TRY(c, hipEventRecord(sl.done, st));
        if (rs != FP_OK) {
            (void)hipStreamSynchronize(st);
            return rs;
        }
    }
    t0 = Clock::now();
    HIP_TRY(c, hipStreamSynchronize(st));
    wait_ms += ms_since(t0);
    if (stats) {
        stats->n_records = total;
        stats->n_chunks = n_chunks;
        stats->max_chunk = max_chunk;
        stats->count_ms = count_ms;
        stats->fill_ms = fill_ms;
        stats->wait_ms = wait_ms;
        stats->total_ms = ms_since(t_call);
    }
    return FP_OK;
}
