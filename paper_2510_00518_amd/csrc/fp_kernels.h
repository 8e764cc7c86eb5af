// Device kernels of libfp (gfx950).  Included once, by fp_lib.hip.
//
// Data layout in HBM (all owned by the context unless noted):
//   omega  f64 [n_modes]                 g = iq*nb + j
//   evec   f64x2 [n_modes][nb]           branch-major within a q-point
//   occ    f64 [n_T][n_modes]            Bose-Einstein occupation per temperature
//   roots  f64x2 [L]                     exp(2 pi i k / L), L = lcm(N0, N1, N2)
//   ifc    f64 [n_terms][3^m]            phi * eV / sqrt(prod M), terms sorted by
//                                        phase key (see below)
//          i32 [n_terms][4]              C (3): phase vector of the mode's own q; a0
//          i32 [n_keys][8]               first term, phase vectors A (3), B (3), term count
//          i32 [n_groups][8]             atoms b, c, d, first key, end key
//   phit   f64x2 [rows][n_keys][3^(m-1)] force constants contracted with the
//                                        row mode's eigenvector and q-phase,
//                                        summed over the terms of each key
//   units  {start, row, count}           work units: <= U consecutive records of one row
//   partial f64 [units][2][n_T]          per-unit sums of Gamma and WP terms
//
// Matrix element with the momentum constraint eliminated (Q_last fixed by
// q + sum Q = 0 mod G), for order 4:
//   V = sum_t exp(2 pi i (Q1.A_t + Q2.B_t + q.C_t)/L) sum_{beta gamma delta}
//       phit_t[beta gamma delta] eps1(b_t)_beta eps2(c_t)_gamma eps3(d_t)_delta
// with A_t = R1 - R3, B_t = R2 - R3, C_t = -R3 (each scaled by L/N_d, mod L);
// order 3 uses A_t = R1 - R2, C_t = -R2.  The q.C_t phase and the contraction
// with e_lambda are folded into phit once per row.  Terms with the same partner
// atoms and the same (A, B) -- a phase key -- share the phase of every process,
// so their folded tables are summed into one entry per key and every kernel
// after the fold runs over keys.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fpk {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kXcd = 8;          // MI355X: 8 accelerator complex dies, blocks dealt round-robin
constexpr int kMaxRoots = 1024;

typedef double d4 __attribute__((ext_vector_type(4)));  // MFMA f64 accumulator tile

struct RowInfo {
    const uint64_t* rec;  // list record array
    int64_t beg, end;     // record range of the row
    int64_t hbase;        // index of the list's first record among all records of the call
    int32_t mode;         // global mode of lambda, -1 if the row is invalid
    int32_t type;         // fp_ptype
};

struct UnitDesc {
    int64_t start;  // first record index
    int32_t row;    // global row, -1 for padding units
    int32_t count;  // records in the unit
};

struct ListArg {
    int32_t type;
    int32_t pad;
    int64_t n_rows, row_base, n_rec, rec_base;
    int64_t rec_shift;  // subtracted from row_off (a row range of a longer list; rec already shifted)
    const int32_t* row_mode;
    const int64_t* row_off;
    const uint64_t* rec;
};

struct ListsArg {
    int32_t n_lists;
    int32_t pad;
    int64_t total_rows;
    ListArg l[8];
};

struct Temps {
    double x[8];  // hbar / (kB T)
};

__device__ inline void raise_flag(int* flag) { atomicOr(flag, 1); }

// Orders LDS writes and reads between the lanes of one wave (the staging areas
// are per wave).  A wave's LDS operations complete in issue order, so waiting
// for its LDS counter suffices; outstanding global loads stay in flight (a
// workgroup-scope fence would also wait for them).  0xC07F = s_waitcnt
// lgkmcnt(0) with vmcnt and expcnt at their maxima (gfx9 encoding).
__device__ inline void lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- utilities

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// P[g] = (v_g . b_0 / N_0, v_g . b_1 / N_1, v_g . b_2 / N_2, 0): the projections
// behind the adaptive width (b = reciprocal vectors as rows)
struct RecipN {
    double b[9];
    double inv_n[3];
};

// proj[g] = (v_g . b_0 / N_0, v_g . b_1 / N_1, v_g . b_2 / N_2, omega_g): the
// frequency rides in the fourth slot so that one 32-byte row holds all a
// width evaluation needs of a mode
__global__ void k_proj(const double* __restrict__ vel, const double* __restrict__ omega, int64_t n_modes, RecipN r,
                       double* __restrict__ proj) {
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_modes;
         g += (int64_t)gridDim.x * blockDim.x) {
        const double v0 = vel[g * 3], v1 = vel[g * 3 + 1], v2 = vel[g * 3 + 2];
        double4 p;
        p.x = (v0 * r.b[0] + v1 * r.b[1] + v2 * r.b[2]) * r.inv_n[0];
        p.y = (v0 * r.b[3] + v1 * r.b[4] + v2 * r.b[5]) * r.inv_n[1];
        p.z = (v0 * r.b[6] + v1 * r.b[7] + v2 * r.b[8]) * r.inv_n[2];
        p.w = omega[g];
        reinterpret_cast<double2*>(proj)[g * 2] = make_double2(p.x, p.y);
        reinterpret_cast<double2*>(proj)[g * 2 + 1] = make_double2(p.z, p.w);
    }
}

__global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// n[T][g] = 1/expm1(hbar w / kB T); inactive modes get 0 (never referenced by valid lists)
__global__ void k_occ(const double* __restrict__ omega, int64_t n_modes, int32_t n_T, Temps t, double floor_,
                      double* __restrict__ occ) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_modes * n_T;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = i % n_modes;
        const int it = (int)(i / n_modes);
        const double w = omega[g];
        occ[i] = w >= floor_ ? 1.0 / expm1(t.x[it] * w) : 0.0;
    }
}

// ------------------------------------------------------------- work units

// One thread per global row: validate the CSR row and count its units.
__global__ void k_rows(ListsArg la, int64_t n_modes, int64_t unit, RowInfo* __restrict__ rows,
                       int64_t* __restrict__ row_units, int* flag) {
    for (int64_t gr = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gr < la.total_rows;
         gr += (int64_t)gridDim.x * blockDim.x) {
        int l = 0;
        while (l + 1 < la.n_lists && gr >= la.l[l + 1].row_base) ++l;
        const ListArg& L = la.l[l];
        const int64_t r = gr - L.row_base;
        int64_t beg = L.row_off[r] - L.rec_shift, end = L.row_off[r + 1] - L.rec_shift;
        int32_t mode = L.row_mode[r];
        bool ok = beg >= 0 && end >= beg && end <= L.n_rec && mode >= 0 && mode < n_modes;
        if (!ok) {
            raise_flag(flag);
            beg = end = 0;
            mode = -1;
        }
        RowInfo ri;
        ri.rec = L.rec;
        ri.hbase = L.rec_base;
        ri.beg = beg;
        ri.end = end;
        ri.mode = mode;
        ri.type = L.type;
        rows[gr] = ri;
        row_units[gr] = (end - beg + unit - 1) / unit;
    }
}

// Exclusive prefix sum of row_units into unit_off[0..n]; one block.
__global__ void k_scan(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ out) {
    __shared__ int64_t part[kBlock];
    const int tid = threadIdx.x;
    const int64_t chunk = (n + kBlock - 1) / kBlock;
    const int64_t b = tid * chunk, e = b + chunk < n ? b + chunk : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t run = 0;
        for (int i = 0; i < kBlock; ++i) {
            const int64_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    int64_t run = part[tid];
    for (int64_t i = b; i < e; ++i) {
        out[i] = run;
        run += in[i];
    }
    if (tid == kBlock - 1) out[n] = run;
}

__global__ void k_units(const int64_t* __restrict__ unit_off, int64_t n_rows, const RowInfo* __restrict__ rows,
                        int64_t unit, int64_t n_units_max, UnitDesc* __restrict__ units) {
    const int64_t total = unit_off[n_rows];
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n_units_max;
         u += (int64_t)gridDim.x * blockDim.x) {
        UnitDesc d;
        if (u >= total) {
            d.start = 0;
            d.row = -1;
            d.count = 0;
        } else {
            int64_t lo = 0, hi = n_rows;  // unit_off[lo] <= u < unit_off[hi]
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (unit_off[mid] <= u) lo = mid; else hi = mid;
            }
            const RowInfo ri = rows[lo];
            d.start = ri.beg + (u - unit_off[lo]) * unit;
            const int64_t left = ri.end - d.start;
            d.row = (int32_t)lo;
            d.count = (int32_t)(left < unit ? left : unit);
        }
        units[u] = d;
    }
}

// ------------------------------------------------------- force constants

// phi_s[t'][c] = phi[perm[t']][c] * scale[t']  (sorted, unit-converted, mass-scaled)
__global__ void k_ifc_scale(const double* __restrict__ phi, const int32_t* __restrict__ perm,
                            const double* __restrict__ scale, int64_t n_terms, int32_t ncomp,
                            double* __restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_terms * ncomp;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i / ncomp;
        const int c = (int)(i % ncomp);
        out[i] = phi[(int64_t)perm[t] * ncomp + c] * scale[t];
    }
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline uint32_t mod_l(uint32_t k, uint32_t L, uint32_t magic) {
    // magic = floor(2^32 / L): the quotient estimate is at most one short
    const uint32_t q = __umulhi(k, magic);
    uint32_t r = k - q * L;
    return r >= L ? r - L : r;
}

struct ModeGeom {
    int32_t N0, N1, N2, nb;
    int32_t L;
    uint32_t magic;
    int32_t s0, s1, s2;        // L / N_d
    uint32_t m_nb, m_n2, m_n12;  // floor((2^32 - 1) / d) for d = nb, N2, N1 N2 (udivm)
};

// x / d for any x < 2^32, with m = floor((2^32 - 1) / d): x m / 2^32 falls short
// of x / d by x (1 + e) / (d 2^32) < 1 (m d = 2^32 - 1 - e, e < d), so the high
// product is the quotient or one less, and one remainder test fixes it.
__device__ inline uint32_t udivm(uint32_t x, uint32_t d, uint32_t m) {
    const uint32_t q = __umulhi(x, m);
    return x - q * d >= d ? q + 1 : q;
}

// q-point index -> mesh coordinates (n0, n1, n2), iq = (n0 N1 + n1) N2 + n2
__device__ inline void q_coords(int32_t iq, const ModeGeom& geo, int32_t& n0, int32_t& n1, int32_t& n2) {
    const uint32_t n12 = (uint32_t)(geo.N1 * geo.N2);
    const uint32_t a = udivm((uint32_t)iq, n12, geo.m_n12);
    const uint32_t r = (uint32_t)iq - a * n12;
    const uint32_t b = udivm(r, (uint32_t)geo.N2, geo.m_n2);
    n0 = (int32_t)a;
    n1 = (int32_t)b;
    n2 = (int32_t)(r - b * (uint32_t)geo.N2);
}

// q-point of global mode g
__device__ inline int32_t mode_q(int32_t g, const ModeGeom& geo) {
    return (int32_t)udivm((uint32_t)g, (uint32_t)geo.nb, geo.m_nb);
}

// phit[row][k][c] = sum_{t in key k} exp(2 pi i q.C_t / L) sum_alpha phi_s[t][alpha][c] e_lambda(a0_t)_alpha
template <int M>
__global__ void k_precontract(const RowInfo* __restrict__ rows, int64_t n_rows, const double2* __restrict__ evec,
                              const double2* __restrict__ roots, ModeGeom geo, const double* __restrict__ phi_s,
                              const int32_t* __restrict__ tmeta, const int32_t* __restrict__ tc, int64_t n_keys,
                              double2* __restrict__ phit) {
    constexpr int NC = M == 3 ? 9 : 27;
    const int64_t total = n_rows * n_keys * NC;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i % NC);
        const int64_t k = (i / NC) % n_keys;
        const int64_t r = i / (NC * n_keys);
        const int32_t g = rows[r].mode;
        double2 acc = make_double2(0.0, 0.0);
        if (g >= 0) {
            const int32_t iq = g / geo.nb;
            const int32_t n2 = iq % geo.N2, n1 = (iq / geo.N2) % geo.N1, n0 = iq / (geo.N1 * geo.N2);
            const int32_t t0 = tmeta[k * 8], t1 = t0 + tmeta[k * 8 + 7];
            for (int32_t t = t0; t < t1; ++t) {
                const int32_t* tt = tc + (int64_t)t * 4;
                const double* p = phi_s + (int64_t)t * (NC * 3);
                const double2* e = evec + (int64_t)g * geo.nb + 3 * tt[3];
                double2 s = make_double2(0.0, 0.0);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double f = p[a * NC + c];
                    const double2 ev = e[a];
                    s.x += f * ev.x;
                    s.y += f * ev.y;
                }
                const uint32_t kq = (uint32_t)(n0 * tt[0] + n1 * tt[1] + n2 * tt[2]);
                s = cmul(roots[mod_l(kq, geo.L, geo.magic)], s);
                acc.x += s.x;
                acc.y += s.y;
            }
        }
        phit[i] = acc;
    }
}

// --------------------------------------------------------------- the rates

// Width of the Gaussian delta.  proj == nullptr: the fixed width (inv_sigma2 =
// 1/sigma^2, gnorm = 1/(sigma sqrt(pi))).  Otherwise the per-process width
// sigma_p = max(factor * sigma0_p, floor_) with sigma0_p^2 the sum over partner
// pairs of |P_i - P_j|^2 divided by 3 (m - 1), where P_g[d] = v_g . b_d / N_d is
// the per-mode projection table (4 doubles per mode, the last unused).
struct Broad {
    double inv_sigma2, gnorm;
    const double* proj;
    double factor, floor_;
};

struct RatesArgs {
    int64_t n_units;
    int64_t n_modes;
    int32_t n_keys, n_groups;  // phase keys (entries of the per-row tables), partner groups
    int32_t n_T;
    int32_t ppl;  // records per lane per unit
    ModeGeom geo;
    Broad br;
    // three-phonon event lists: the contributions of each record to its two
    // partner modes, scaled by the final prefactors, go to ev_val[(2 rec + slot)
    // * 2 n_T + {it, n_T + it}] with the target mode in ev_key[2 rec + slot]
    // (slot 0: the 3+ partner, slot 1: the 3- product; 0x7FFFFFFF for none),
    // rec being the record's index among all records of the call; k_event_reduce
    // adds them per mode in a fixed order
    double pref, wpref;
    double* ev_val;
    int32_t* ev_key;
};

// Pointers travel as separate restrict-qualified arguments so that the compiler
// can prove the wave-uniform tables (phit, tmeta, groups, rows, units) are never
// written during the kernel and fetch them with scalar loads.
#define FP_RATES_PARAMS                                                                                       \
    const double* __restrict__ omega, const double2* __restrict__ evec, const double* __restrict__ occ,      \
        const double2* __restrict__ roots, const double2* __restrict__ phit, const int32_t* __restrict__ tmeta, \
        const int32_t* __restrict__ groups, const RowInfo* __restrict__ rows,                                  \
        const UnitDesc* __restrict__ units, double* __restrict__ partial, int* __restrict__ flag, RatesArgs a

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ inline void type_signs(int type, int& s1, int& s2, int& s3) {
    // 3ph: s1, s2; 4ph: s1, s2, s3 (slot 0 is +1)
    switch (type) {
        case 0: s1 = 1; s2 = -1; s3 = 0; break;    // 3+
        case 1: s1 = -1; s2 = -1; s3 = 0; break;   // 3-
        case 5: s1 = 1; s2 = -1; s3 = 0; break;    // 3ph event, as 3+
        case 2: s1 = 1; s2 = 1; s3 = -1; break;    // ++
        case 3: s1 = 1; s2 = -1; s3 = -1; break;   // +-
        default: s1 = -1; s2 = -1; s3 = -1; break; // --
    }
}

__device__ inline int wrapn(int x, int n) {
    // x mod n for x in (-4n, 4n) (every caller passes a sum of at most three
    // mesh coordinates, signed): two folds by 2n, then one by n
    x = x < 0 ? x + 2 * n : x;
    x = x < 0 ? x + 2 * n : x;
    x = x >= 2 * n ? x - 2 * n : x;
    return x >= n ? x - n : x;
}

// One listed process as seen by one lane: partner modes, signed partner
// wavevectors (mesh integers), and the weight w G(Delta)/prod(omega).  An empty
// slot (past the end of the unit, or a record outside the mesh) points every
// index at the row's own mode and carries weight 0, so the uniform loops below
// read only valid memory and add nothing.
struct Proc {
    int32_t g1, g2, gl;
    int32_t Q10, Q11, Q12, Q20, Q21, Q22;
    double base;
};

// Index part of setup_proc for an order-4 record: partner modes and signed
// wavevectors, no frequencies or weight (base = 0).  Invalid or empty slots
// point at the row's mode, like setup_proc.
__device__ inline Proc decode4(bool have, uint64_t rec, int s1, int s2, int s3, int32_t g0, int32_t c00, int32_t c01,
                               int32_t c02, const ModeGeom& geo, int64_t n_modes, int* __restrict__ flag) {
    Proc p;
    p.g1 = p.g2 = p.gl = g0;
    p.Q10 = p.Q11 = p.Q12 = p.Q20 = p.Q21 = p.Q22 = 0;
    p.base = 0.0;
    if (!have) return p;
    const int nb = geo.nb;
    const int32_t g1 = (int32_t)(rec & 0xFFFFFFu);
    const int32_t g2 = (int32_t)((rec >> 24) & 0xFFFFFFu);
    const int32_t j_last = (int32_t)((rec >> 48) & 0xFFu);
    if (g1 >= n_modes || g2 >= n_modes || j_last >= nb) {
        raise_flag(flag);
        return p;
    }
    int32_t c10, c11, c12, c20, c21, c22;
    q_coords(mode_q(g1, geo), geo, c10, c11, c12);
    q_coords(mode_q(g2, geo), geo, c20, c21, c22);
    p.Q10 = s1 > 0 ? c10 : wrapn(-c10, geo.N0);
    p.Q11 = s1 > 0 ? c11 : wrapn(-c11, geo.N1);
    p.Q12 = s1 > 0 ? c12 : wrapn(-c12, geo.N2);
    p.Q20 = s2 > 0 ? c20 : wrapn(-c20, geo.N0);
    p.Q21 = s2 > 0 ? c21 : wrapn(-c21, geo.N1);
    p.Q22 = s2 > 0 ? c22 : wrapn(-c22, geo.N2);
    int32_t ql0 = wrapn(-(c00 + p.Q10 + p.Q20), geo.N0);
    int32_t ql1 = wrapn(-(c01 + p.Q11 + p.Q21), geo.N1);
    int32_t ql2 = wrapn(-(c02 + p.Q12 + p.Q22), geo.N2);
    if (s3 < 0) {
        ql0 = wrapn(-ql0, geo.N0);
        ql1 = wrapn(-ql1, geo.N1);
        ql2 = wrapn(-ql2, geo.N2);
    }
    p.g1 = g1;
    p.g2 = g2;
    p.gl = ((ql0 * geo.N1 + ql1) * geo.N2 + ql2) * nb + j_last;
    return p;
}

// pm[iq] = (max over the branches j of |proj[iq nb + j][d]|, d = 0, 1, 2; 0)
__global__ void k_proj_max(const double* __restrict__ proj, int64_t nq, int nb, double* __restrict__ pm) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nq; q += (int64_t)gridDim.x * blockDim.x) {
        double m[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < nb; ++j)
            for (int d = 0; d < 3; ++d) m[d] = fmax(m[d], fabs(proj[(q * nb + j) * 4 + d]));
        for (int d = 0; d < 3; ++d) pm[q * 4 + d] = m[d];
        pm[q * 4 + 3] = 0.0;
    }
}

// one mode's row of the projection table: (proj_0, proj_1, proj_2, omega)
struct Proj4 {
    double2 a, b;
};
__device__ inline Proj4 ld_proj4(const double* __restrict__ proj, int32_t g) {
    Proj4 p;
    p.a = *reinterpret_cast<const double2*>(proj + (size_t)g * 4);
    p.b = *reinterpret_cast<const double2*>(proj + (size_t)g * 4 + 2);
    return p;
}
// the same squared distance as proj_sq, from rows already loaded
__device__ inline double proj_sq4(const Proj4& x, const Proj4& y) {
    const double d0 = x.a.x - y.a.x, d1 = x.a.y - y.a.y, d2 = x.b.x - y.b.x;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

// squared distance of two projection rows (three directions)
__device__ inline double proj_sq(const double* __restrict__ proj, int32_t gi, int32_t gj) {
    const double2 a01 = *reinterpret_cast<const double2*>(proj + (size_t)gi * 4);
    const double2 b01 = *reinterpret_cast<const double2*>(proj + (size_t)gj * 4);
    const double a2 = proj[(size_t)gi * 4 + 2], b2 = proj[(size_t)gj * 4 + 2];
    const double d0 = a01.x - b01.x, d1 = a01.y - b01.y, d2 = a2 - b2;
    return d0 * d0 + d1 * d1 + d2 * d2;
}

template <int M>
__device__ inline Proc setup_proc(bool have, uint64_t rec, int type, int s1, int s2, int s3, int32_t g0, int32_t c00,
                                  int32_t c01, int32_t c02, double w0, const ModeGeom& geo,
                                  const double* __restrict__ omega, int64_t n_modes, int* __restrict__ flag,
                                  const Broad& br) {
    Proc p;
    p.g1 = p.g2 = p.gl = g0;
    p.Q10 = p.Q11 = p.Q12 = p.Q20 = p.Q21 = p.Q22 = 0;
    p.base = 0.0;
    if (!have) return p;
    const int nb = geo.nb;
    const int32_t g1 = (int32_t)(rec & 0xFFFFFFu);
    int32_t g2, j_last;
    if (M == 3) {
        g2 = 0;
        j_last = (int32_t)((rec >> 24) & 0xFFu);
    } else {
        g2 = (int32_t)((rec >> 24) & 0xFFFFFFu);
        j_last = (int32_t)((rec >> 48) & 0xFFu);
    }
    if (g1 >= n_modes || g2 >= n_modes || j_last >= nb) {
        raise_flag(flag);
        return p;
    }
    // signed wavevectors of the listed partners; the last partner follows from momentum
    int32_t c10, c11, c12;
    q_coords(mode_q(g1, geo), geo, c10, c11, c12);
    p.Q10 = s1 > 0 ? c10 : wrapn(-c10, geo.N0);
    p.Q11 = s1 > 0 ? c11 : wrapn(-c11, geo.N1);
    p.Q12 = s1 > 0 ? c12 : wrapn(-c12, geo.N2);
    if (M == 4) {
        int32_t c20, c21, c22;
        q_coords(mode_q(g2, geo), geo, c20, c21, c22);
        p.Q20 = s2 > 0 ? c20 : wrapn(-c20, geo.N0);
        p.Q21 = s2 > 0 ? c21 : wrapn(-c21, geo.N1);
        p.Q22 = s2 > 0 ? c22 : wrapn(-c22, geo.N2);
    }
    const int sl = M == 3 ? s2 : s3;
    // Q_last = -(q + Q1 (+ Q2)); q_last = s_last * Q_last
    int32_t ql0 = wrapn(-(c00 + p.Q10 + p.Q20), geo.N0);
    int32_t ql1 = wrapn(-(c01 + p.Q11 + p.Q21), geo.N1);
    int32_t ql2 = wrapn(-(c02 + p.Q12 + p.Q22), geo.N2);
    if (sl < 0) {
        ql0 = wrapn(-ql0, geo.N0);
        ql1 = wrapn(-ql1, geo.N1);
        ql2 = wrapn(-ql2, geo.N2);
    }
    const int32_t gl = ((ql0 * geo.N1 + ql1) * geo.N2 + ql2) * nb + j_last;
    const double w1 = omega[g1];
    const double wl = omega[gl];
    const double w2 = M == 4 ? omega[g2] : wl;
    double delta = s1 > 0 ? w0 + w1 : w0 - w1;
    delta = s2 > 0 ? delta + w2 : delta - w2;
    if (M == 4) delta = s3 > 0 ? delta + wl : delta - wl;
    double wprod = w0 * w1 * w2;
    if (M == 4) wprod *= wl;
    // triangle weight from equality of interchangeable partners
    double wt = 1.0;
    if (M == 3) {
        if (type == 1 && g1 == gl) wt = 0.5;
    } else if (type == 2) {
        if (g1 == g2) wt = 0.5;
    } else if (type == 3) {
        if (g2 == gl) wt = 0.5;
    } else {
        const int eq = (g1 == g2) + (g2 == gl) + (g1 == gl);
        wt = eq == 3 ? (1.0 / 6.0) : (eq >= 1 ? 0.5 : 1.0);
    }
    p.g1 = g1;
    p.g2 = M == 4 ? g2 : gl;  // order 3: slot 2 is the momentum-fixed partner
    p.gl = gl;
    double inv_sigma2 = br.inv_sigma2, gnorm = br.gnorm;
    if (br.proj) {
        // partners: g1, gl (order 3); g1, g2, gl (order 4)
        double s2 = proj_sq(br.proj, g1, M == 4 ? g2 : gl);
        if (M == 4) s2 += proj_sq(br.proj, g1, gl) + proj_sq(br.proj, g2, gl);
        const double sig = fmax(br.factor * sqrt(s2 * (M == 3 ? (1.0 / 6.0) : (1.0 / 9.0))), br.floor_);
        inv_sigma2 = 1.0 / (sig * sig);
        gnorm = 0.56418958354775628695 / sig;  // 1/(sigma sqrt(pi))
    }
    p.base = wt * exp(-(delta * delta) * inv_sigma2) * gnorm / wprod;
    return p;
}

__device__ inline double2 cfma(double2 acc, double2 a, double2 b) {
    acc.x += a.x * b.x;
    acc.x -= a.y * b.y;
    acc.y += a.x * b.y;
    acc.y += a.y * b.x;
    return acc;
}

__device__ inline double2 ld_eps(const double2* __restrict__ e, double csign) {
    double2 v = *e;
    v.y *= csign;
    return v;
}

// Contraction variants (wave-uniform force-constant stream, per-lane eigenvectors):
//   CT = 0  P-form: P = eps1 (x) eps2 (x) eps3 once per partner-atom group, then
//           27 complex MACs + 1 phase MAC per term (order 4; order 3: 9 + 1)
//   CT = 1  W-form: w = eps2 (x) eps3 per group, then per term 27 MACs into three
//           partial sums u_beta, 3 MACs with eps1, 1 phase MAC (order 4 only);
//           a third of the P-form's registers for 3 more MACs per term
// NP processes per lane are evaluated together, so every scalar-loaded
// force-constant value feeds NP times as many FMAs.
template <int M, int MAXT, int CT, int NP, int WAVES>
__global__ __launch_bounds__(kBlock, WAVES) void k_rates(FP_RATES_PARAMS) {
    constexpr int NC = M == 3 ? 9 : 27;
    __shared__ double2 sroots[kMaxRoots];
    for (int i = threadIdx.x; i < a.geo.L; i += kBlock) sroots[i] = roots[i];
    __syncthreads();

    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Blocks are dealt to the dies round-robin; give each die a contiguous range
    // of units so consecutive units of one row share that die's L2.
    const int xcd = blockIdx.x % kXcd;
    const int64_t per_xcd = (a.n_units + kXcd - 1) / kXcd;
    const int64_t u_beg = xcd * per_xcd;
    const int64_t u_end = u_beg + per_xcd < a.n_units ? u_beg + per_xcd : a.n_units;
    const int64_t wstride = (int64_t)(gridDim.x / kXcd) * kWavesPerBlock;
    const ModeGeom geo = a.geo;
    const int nb = geo.nb;

    for (int64_t u = u_beg + (int64_t)(blockIdx.x / kXcd) * kWavesPerBlock + wave; u < u_end; u += wstride) {
        const UnitDesc ud = units[u];
        const int32_t row = __builtin_amdgcn_readfirstlane(ud.row);
        const int32_t count = __builtin_amdgcn_readfirstlane(ud.count);
        double accg[MAXT], accw[MAXT];
#pragma unroll
        for (int it = 0; it < MAXT; ++it) accg[it] = accw[it] = 0.0;
        if (row >= 0 && count > 0) {
            const RowInfo ri = rows[row];
            const int32_t g0 = __builtin_amdgcn_readfirstlane(ri.mode);
            const int type = __builtin_amdgcn_readfirstlane(ri.type);
            int s1, s2, s3;
            type_signs(type, s1, s2, s3);
            const int sl = M == 3 ? s2 : s3;
            const double c1 = s1 > 0 ? 1.0 : -1.0;
            const double c2 = s2 > 0 ? 1.0 : -1.0;
            const double c3 = sl > 0 ? 1.0 : -1.0;
            const int32_t iq0 = g0 / nb;
            const int32_t c00 = iq0 / (geo.N1 * geo.N2), c01 = (iq0 / geo.N2) % geo.N1, c02 = iq0 % geo.N2;
            const double w0 = omega[g0];
            const double2* __restrict__ phit_row = phit + (int64_t)row * a.n_keys * NC;
            for (int p0 = 0; p0 * kWave < count; p0 += NP) {
                Proc pr[NP];
                uint32_t evf[NP];  // event flags (FP_3E records): bit 0 the 3+ processes, bit 1 the 3- one
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    const int idx = (p0 + i) * kWave + lane;
                    const bool have = idx < count && p0 + i < a.ppl;
                    const uint64_t rec = have ? ri.rec[ud.start + idx] : 0;
                    pr[i] = setup_proc<M>(have, rec, type, s1, s2, s3, g0, c00, c01, c02, w0, geo, omega, a.n_modes,
                                          flag, a.br);
                    const bool valid = (int64_t)(rec & 0xFFFFFFu) < a.n_modes && (int32_t)((rec >> 24) & 0xFFu) < nb;
                    evf[i] = (M == 3 && type == 5 && have && valid) ? (uint32_t)(rec >> 32) & 3u : 0u;
                }
                double2 V[NP];
#pragma unroll
                for (int i = 0; i < NP; ++i) V[i] = make_double2(0.0, 0.0);
                for (int gi = 0; gi < a.n_groups; ++gi) {
                    const int32_t* G = groups + gi * 8;
                    const int32_t ab = G[0], ac = G[1], ad = G[2], t0 = G[3], t1 = G[4];
                    if (M == 3) {
                        double2 P[NP][9];
#pragma unroll
                        for (int i = 0; i < NP; ++i) {
                            const double2* e1 = evec + (int64_t)pr[i].g1 * nb + 3 * ab;
                            const double2* e2 = evec + (int64_t)pr[i].g2 * nb + 3 * ac;
                            double2 x[3], y[3];
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                x[k] = ld_eps(e1 + k, c1);
                                y[k] = ld_eps(e2 + k, c2);
                            }
#pragma unroll
                            for (int b = 0; b < 3; ++b)
#pragma unroll
                                for (int c = 0; c < 3; ++c) P[i][b * 3 + c] = cmul(x[b], y[c]);
                        }
                        for (int t = t0; t < t1; ++t) {
                            const int32_t* tm = tmeta + t * 8;
                            const double2* F = phit_row + (int64_t)t * 9;
                            double2 sacc[NP];
#pragma unroll
                            for (int i = 0; i < NP; ++i) sacc[i] = make_double2(0.0, 0.0);
#pragma unroll
                            for (int c = 0; c < 9; ++c) {
                                const double2 f = F[c];
#pragma unroll
                                for (int i = 0; i < NP; ++i) sacc[i] = cfma(sacc[i], f, P[i][c]);
                            }
#pragma unroll
                            for (int i = 0; i < NP; ++i) {
                                const uint32_t k = (uint32_t)(pr[i].Q10 * tm[1] + pr[i].Q11 * tm[2] + pr[i].Q12 * tm[3]);
                                V[i] = cfma(V[i], sroots[mod_l(k, geo.L, geo.magic)], sacc[i]);
                            }
                        }
                    } else if (CT == 0) {
                        double2 P[NP][27];
#pragma unroll
                        for (int i = 0; i < NP; ++i) {
                            const double2* e1 = evec + (int64_t)pr[i].g1 * nb + 3 * ab;
                            const double2* e2 = evec + (int64_t)pr[i].g2 * nb + 3 * ac;
                            const double2* e3 = evec + (int64_t)pr[i].gl * nb + 3 * ad;
                            double2 x[3], y[3], z[3];
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                x[k] = ld_eps(e1 + k, c1);
                                y[k] = ld_eps(e2 + k, c2);
                                z[k] = ld_eps(e3 + k, c3);
                            }
#pragma unroll
                            for (int b = 0; b < 3; ++b)
#pragma unroll
                                for (int c = 0; c < 3; ++c) {
                                    const double2 xy = cmul(x[b], y[c]);
#pragma unroll
                                    for (int d = 0; d < 3; ++d) P[i][(b * 3 + c) * 3 + d] = cmul(xy, z[d]);
                                }
                        }
                        for (int t = t0; t < t1; ++t) {
                            const int32_t* tm = tmeta + t * 8;
                            const double2* F = phit_row + (int64_t)t * 27;
                            double2 sa[NP], sb[NP];
#pragma unroll
                            for (int i = 0; i < NP; ++i) sa[i] = sb[i] = make_double2(0.0, 0.0);
#pragma unroll
                            for (int c = 0; c < 27; ++c) {
                                const double2 f = F[c];
#pragma unroll
                                for (int i = 0; i < NP; ++i) {
                                    if (c & 1) sb[i] = cfma(sb[i], f, P[i][c]);
                                    else sa[i] = cfma(sa[i], f, P[i][c]);
                                }
                            }
#pragma unroll
                            for (int i = 0; i < NP; ++i) {
                                const uint32_t k = (uint32_t)(pr[i].Q10 * tm[1] + pr[i].Q11 * tm[2] + pr[i].Q12 * tm[3] +
                                                              pr[i].Q20 * tm[4] + pr[i].Q21 * tm[5] + pr[i].Q22 * tm[6]);
                                const double2 s = make_double2(sa[i].x + sb[i].x, sa[i].y + sb[i].y);
                                V[i] = cfma(V[i], sroots[mod_l(k, geo.L, geo.magic)], s);
                            }
                        }
                    } else {
                        double2 x[NP][3], w[NP][9];
#pragma unroll
                        for (int i = 0; i < NP; ++i) {
                            const double2* e1 = evec + (int64_t)pr[i].g1 * nb + 3 * ab;
                            const double2* e2 = evec + (int64_t)pr[i].g2 * nb + 3 * ac;
                            const double2* e3 = evec + (int64_t)pr[i].gl * nb + 3 * ad;
                            double2 y[3], z[3];
#pragma unroll
                            for (int k = 0; k < 3; ++k) {
                                x[i][k] = ld_eps(e1 + k, c1);
                                y[k] = ld_eps(e2 + k, c2);
                                z[k] = ld_eps(e3 + k, c3);
                            }
#pragma unroll
                            for (int c = 0; c < 3; ++c)
#pragma unroll
                                for (int d = 0; d < 3; ++d) w[i][c * 3 + d] = cmul(y[c], z[d]);
                        }
                        for (int t = t0; t < t1; ++t) {
                            const int32_t* tm = tmeta + t * 8;
                            const double2* F = phit_row + (int64_t)t * 27;
                            double2 s[NP];
#pragma unroll
                            for (int i = 0; i < NP; ++i) s[i] = make_double2(0.0, 0.0);
#pragma unroll
                            for (int b = 0; b < 3; ++b) {
                                double2 uu[NP];
#pragma unroll
                                for (int i = 0; i < NP; ++i) uu[i] = make_double2(0.0, 0.0);
#pragma unroll
                                for (int c = 0; c < 9; ++c) {
                                    const double2 f = F[b * 9 + c];
#pragma unroll
                                    for (int i = 0; i < NP; ++i) uu[i] = cfma(uu[i], f, w[i][c]);
                                }
#pragma unroll
                                for (int i = 0; i < NP; ++i) s[i] = cfma(s[i], uu[i], x[i][b]);
                            }
#pragma unroll
                            for (int i = 0; i < NP; ++i) {
                                const uint32_t k = (uint32_t)(pr[i].Q10 * tm[1] + pr[i].Q11 * tm[2] + pr[i].Q12 * tm[3] +
                                                              pr[i].Q20 * tm[4] + pr[i].Q21 * tm[5] + pr[i].Q22 * tm[6]);
                                V[i] = cfma(V[i], sroots[mod_l(k, geo.L, geo.magic)], s[i]);
                            }
                        }
                    }
                }

                // ---- three-phonon events: one matrix element for all three modes;
                // the partners' rates go to the call's event buffers (k_event_reduce)
                if (M == 3 && type == 5) {
#pragma unroll
                    for (int i = 0; i < NP; ++i) {
                        const int idx = (p0 + i) * kWave + lane;
                        if (!(idx < count && p0 + i < a.ppl)) continue;
                        const int64_t rg = ri.hbase + ud.start + idx;  // record index in the call
                        const double V2 = V[i].x * V[i].x + V[i].y * V[i].y;
                        const int32_t gb = pr[i].g1, gc = pr[i].gl;
                        const double wb = omega[gb], wc = omega[gc];
                        // the 3- process of g'': mismatch (w'' - w) - w', weight 1/2 if g' == g
                        const double dm = (wc - w0) - wb;
                        const double bm = (gb == g0 ? 0.5 : 1.0) * exp(-(dm * dm) * a.br.inv_sigma2) * a.br.gnorm /
                                          (w0 * wb * wc);
                        const bool to_b = (evf[i] & 1u) && gb != g0, to_c = (evf[i] & 2u) != 0u;
                        double* vb = a.ev_val + (2 * rg) * (2 * a.n_T);
                        double* vc = vb + 2 * a.n_T;
#pragma unroll
                        for (int it = 0; it < MAXT; ++it) {
                            if (it < a.n_T) {
                                const double* n = occ + (int64_t)it * a.n_modes;
                                const double na = n[g0], nb_ = n[gb], nc = n[gc];
                                if (evf[i] & 1u) {
                                    const double xa = pr[i].base * (nb_ - nc);
                                    accw[it] += xa;
                                    accg[it] += xa * V2;
                                }
                                const double xb = pr[i].base * (na - nc);
                                const double xc = bm * (1.0 + na + nb_);
                                vb[it] = to_b ? a.pref * xb * V2 : 0.0;
                                vb[a.n_T + it] = to_b ? a.wpref * xb : 0.0;
                                vc[it] = to_c ? a.pref * xc * V2 : 0.0;
                                vc[a.n_T + it] = to_c ? a.wpref * xc : 0.0;
                            }
                        }
                        a.ev_key[2 * rg] = to_b ? gb : 0x7FFFFFFF;
                        a.ev_key[2 * rg + 1] = to_c ? gc : 0x7FFFFFFF;
                    }
                    continue;
                }
                // ---- occupation per temperature
#pragma unroll
                for (int i = 0; i < NP; ++i) {
                    const double V2 = V[i].x * V[i].x + V[i].y * V[i].y;
#pragma unroll
                    for (int it = 0; it < MAXT; ++it) {
                        if (it < a.n_T) {
                            const double* n = occ + (int64_t)it * a.n_modes;
                            const double n1 = n[pr[i].g1], nl = n[pr[i].gl];
                            double oc;
                            if (M == 3) {
                                oc = type == 0 ? n1 - nl : 1.0 + n1 + nl;
                            } else {
                                const double n2 = n[pr[i].g2];
                                if (type == 2)
                                    oc = n1 * n2 * (1.0 + nl) - (1.0 + n1) * (1.0 + n2) * nl;
                                else if (type == 3)
                                    oc = n1 * (1.0 + n2) * (1.0 + nl) - (1.0 + n1) * n2 * nl;
                                else
                                    oc = (1.0 + n1) * (1.0 + n2) * (1.0 + nl) - n1 * n2 * nl;
                            }
                            const double xw = pr[i].base * oc;
                            accw[it] += xw;
                            accg[it] += xw * V2;
                        }
                    }
                }
            }
        }
        double* out = partial + u * (2 * a.n_T);
#pragma unroll
        for (int it = 0; it < MAXT; ++it) {
            if (it < a.n_T) {
                const double sg = wave_sum(accg[it]);
                const double sw = wave_sum(accw[it]);
                if (lane == 0) {
                    out[it] = sg;
                    out[a.n_T + it] = sw;
                }
            }
        }
    }
}

// One block per row of one list: sum the row's unit partials in a fixed tree
// order and add pref * sum into out[T][mode].
__global__ void k_finalize(const double* __restrict__ partial, const int64_t* __restrict__ unit_off,
                           const RowInfo* __restrict__ rows, int64_t row0, int32_t n_T, double pref, double wpref,
                           double* __restrict__ gamma_out, double* __restrict__ wp_out, int64_t n_modes) {
    __shared__ double red[kBlock];
    const int64_t r = row0 + blockIdx.x;
    const int32_t mode = rows[r].mode;
    const int64_t u0 = unit_off[r], u1 = unit_off[r + 1];
    for (int q = 0; q < 2 * n_T; ++q) {
        double s = 0.0;
        for (int64_t u = u0 + threadIdx.x; u < u1; u += kBlock) s += partial[u * (2 * n_T) + q];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0 && mode >= 0) {
            const int it = q < n_T ? q : q - n_T;
            if (q < n_T) {
                if (gamma_out) gamma_out[(int64_t)it * n_modes + mode] += pref * red[0];
            } else {
                if (wp_out) wp_out[(int64_t)it * n_modes + mode] += wpref * red[0];
            }
        }
        __syncthreads();
    }
}

// k_fill for int32
__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// Event contributions to the partner modes, added per mode in the order of the
// stably sorted (mode, entry) pairs: deterministic, whatever the timing of the
// rate kernel.  keys are sorted, idx the entries (2 rec + slot) in that order.
__global__ void k_event_reduce(const int32_t* __restrict__ keys, const int32_t* __restrict__ idx, int64_t n,
                               const double* __restrict__ val, int32_t n_T, double* __restrict__ gamma_out,
                               double* __restrict__ wp_out, int64_t n_modes) {
    for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < n_modes;
         m += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;  // first key >= m
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (keys[mid] < m) lo = mid + 1; else hi = mid;
        }
        for (int it = 0; it < n_T; ++it) {
            double sg = 0.0, sw = 0.0;
            for (int64_t k = lo; k < n && keys[k] == m; ++k) {
                const double* v = val + (int64_t)idx[k] * (2 * n_T);
                sg += v[it];
                sw += v[n_T + it];
            }
            if (lo < n && keys[lo] == m) {
                if (gamma_out) gamma_out[(int64_t)it * n_modes + m] += sg;
                if (wp_out) wp_out[(int64_t)it * n_modes + m] += sw;
            }
        }
    }
}

// --------------------------------------------------------------- kappa_RTA

// One block per temperature: kappa[T][9] and optionally d(tr kappa/3)/dGamma.
__global__ void k_kappa(const int32_t* __restrict__ q1, const double* __restrict__ q1w, int32_t n_q1, int32_t nb,
                        const double* __restrict__ omega, const double* __restrict__ vel,
                        const double* __restrict__ gamma, int64_t n_modes, Temps tx, Temps pref,
                        double floor_, double* __restrict__ kappa, double* __restrict__ dk, int* flag) {
    __shared__ double red[kBlock];
    const int it = blockIdx.x;
    const double x = tx.x[it];
    const double* G = gamma + (int64_t)it * n_modes;
    const int64_t n = (int64_t)n_q1 * nb;
    double acc[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc[k] = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kBlock) {
        const int64_t iq = q1[i / nb];
        if (iq < 0 || iq * nb >= n_modes) {
            raise_flag(flag);
            continue;
        }
        const int64_t g = iq * nb + i % nb;
        const double w = omega[g];
        const double gm = G[g];
        double c = 0.0;
        if (w >= floor_ && gm > 0.0) {
            const double nn = 1.0 / expm1(x * w);
            // n(n+1) (hbar w)^2 / kB T^2 * w_q, with the 1/(kB T^2 N Omega) in pref
            c = q1w[i / nb] * nn * (nn + 1.0) * w * w;
        }
        const double v0 = vel[g * 3], v1 = vel[g * 3 + 1], v2 = vel[g * 3 + 2];
        const double inv = c > 0.0 ? 1.0 / gm : 0.0;
        acc[0] += c * v0 * v0 * inv; acc[1] += c * v0 * v1 * inv; acc[2] += c * v0 * v2 * inv;
        acc[3] += c * v1 * v0 * inv; acc[4] += c * v1 * v1 * inv; acc[5] += c * v1 * v2 * inv;
        acc[6] += c * v2 * v0 * inv; acc[7] += c * v2 * v1 * inv; acc[8] += c * v2 * v2 * inv;
        if (dk) dk[(int64_t)it * n_modes + g] = -pref.x[it] * c * (v0 * v0 + v1 * v1 + v2 * v2) * inv * inv / 3.0;
    }
    for (int k = 0; k < 9; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) kappa[it * 9 + k] = pref.x[it] * red[0];
        __syncthreads();
    }
}

}  // namespace fpk
