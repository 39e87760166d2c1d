// fem_api.cpp -- the C ABI of libfem (declared in include/fem.h): argument validation, the
// per-degree constant tables (built once in FP64, rounded per precision) and kernel dispatch.
#include "fem.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fem_kernel.h"
#include "fem_launch.h"
#include "fem_layout.h"
#include "fem_tables.h"
#include "fem_jacobian.h"
#include "fem_transpose.h"
#include "fem_mixed.h"

static_assert(FEM_NOALLOC_MAX_NEL == fem::NOALLOC_MAX_NEL, "one element capacity of the static scratch");
static_assert(FEM_PRISM(1) == fem::PRISM_BASE + 1, "one numbering of the prism's variant keys");

namespace fem {
hipError_t prepare_f64();
hipError_t prepare_f32();
hipError_t prepare_bf16();
hipError_t prepare_split_bf16();
hipError_t prepare_split_f16();
hipError_t launch_f64(int p, int v, const KArgs &a, hipStream_t s, int64_t cus);
hipError_t launch_f32(int p, int v, const KArgs &a, hipStream_t s, int64_t cus);
hipError_t launch_bf16(int p, int v, const KArgs &a, hipStream_t s, int64_t cus);
hipError_t launch_split_bf16(int p, int v, const KArgs &a, hipStream_t s, int64_t cus);
hipError_t launch_split_f16(int p, int v, const KArgs &a, hipStream_t s, int64_t cus);
hipError_t launch_mixed_f64(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus);
hipError_t launch_mixed_f32(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus);
hipError_t launch_mixed_bf16(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus);
hipError_t launch_mixed_split_bf16(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus);
hipError_t launch_mixed_split_f16(const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus);
int variants_f64(int p);
int variants_f32(int p);
int variants_bf16(int p);
int variants_split_bf16(int p);
int variants_split_f16(int p);
hipError_t field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step,
                         hipStream_t s);
hipError_t gather_sample(int64_t nsel, const int32_t *sel, int32_t nrows, const int32_t *step, int64_t nel,
                         const int64_t *a_off, const int64_t *b_off, const void *A, const void *b,
                         void *out_A, int64_t cap_A, void *out_b, int64_t cap_b, int32_t entry_bytes,
                         hipStream_t s);
void staged_release();
}  // namespace fem

namespace {

using namespace fem;

struct DegreeDev {
    const double *xq = nullptr, *wq = nullptr, *LD64 = nullptr;
    const float *LD32 = nullptr;
    const double *phi64 = nullptr;  // prisms: shape-function values at the points
    const void *row[5][2] = {};
    const void *bcol[3] = {};  // column-operand factor table B per family (FP32, FP32, FP64)
    float c_bound = 0.0f;
};

struct State {
    int device = -1;
    void *blob = nullptr;  // one device allocation holding every table
    DegreeDev deg[18];     // [p]: hexahedra, [PRISM_BASE + p]: prisms
};
// Device address of the static mixed-degree scratch on each device fem_init has run on (taken
// with that device current; every device holds its own copy of the array).
constexpr int MAX_DEVICES = 64;
void *g_scratch[MAX_DEVICES] = {};
State g_state;
std::mutex g_mutex;

int64_t g_cus = 256;  // compute units of the device (persistent grids: CUs x resident WGs)
// Elasticity: how the blocks below the diagonal (the transposes of those above, by the major
// symmetry of c_ijkl) are formed, per degree, for the 16-bit contraction paths and for FP32 /
// FP64: integrated like the others (E_NINE), copied transposed by a separate kernel after the
// six upper blocks (E_COPY), or written transposed by the epilogue of the upper block's own
// launch from the tile it stages anyway (E_EPI, no re-read of the block). Measured on MI355X.
enum ElasticMode { E_NINE = 0, E_COPY = 1, E_EPI = 2 };
constexpr int ELASTIC_MODE_K16[8] = {E_NINE, E_NINE, E_EPI, E_EPI, E_EPI, E_EPI, E_EPI, E_EPI};
constexpr int ELASTIC_MODE_WIDE[8] = {E_NINE, E_NINE, E_EPI, E_EPI, E_EPI, E_EPI, E_EPI, E_EPI};
int elastic_mode(int P, int prec)
{
    const bool wide = prec == FEM_FP64 || prec == FEM_FP32;
    return wide ? ELASTIC_MODE_WIDE[deg_of(P)] : ELASTIC_MODE_K16[deg_of(P)];
}

uint16_t bf16_bits_rne(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
double bf16_value(uint16_t h)
{
    uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return double(f);
}
uint16_t f16_bits(double x)
{
    _Float16 h = (_Float16)x;
    uint16_t b;
    std::memcpy(&b, &h, 2);
    return b;
}
double f16_value(uint16_t b)
{
    _Float16 h;
    std::memcpy(&h, &b, 2);
    return double(h);
}

// Row-operand value of (group g, row block rb, lane, slot v) for family fam, or 0 if padded.
double row_value(const std::vector<double> &B, int p, int fam, int g, int rb, int lane, int v)
{
    const int ns = ns_of(p);
    const int q = slot_point(fam, g, lane, v);
    const int r = slot_comp(v);
    const int i = rb * fam_tm(fam) + lane % fam_tm(fam);
    if (q >= nq_of(p) || i >= ns) return 0.0;
    return B[(size_t(q) * 4 + r) * ns + i];
}

struct HostBlob {
    std::vector<unsigned char> bytes;
    size_t put(const void *src, size_t n)
    {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + n);
        std::memcpy(bytes.data() + off, src, n);
        return off;
    }
};

struct Offs {
    size_t xq = 0, wq = 0, ld64 = 0, ld32 = 0, phi64 = 0, row[5][2] = {}, bcol[3] = {};
    bool has_lo[5] = {}, has_1d = false, has_phi = false;
    float c_bound = 0.0f;
};

// The operand tables of element P (hexahedron p or prism PRISM_BASE + p) from its FP64 reference
// operand B[(q, r)][i]: the column-operand B factors per family and the row operand B^T per
// precision, in the fragment layouts of fem_layout.h.
void put_operand_tables(HostBlob &hb, Offs &o, int P, const std::vector<double> &B)
{
    const int ns = ns_of(P), nq = nq_of(P);
    // B in the column-operand fragment layout of each family: [group][table block][lane][slot]
    // holds B[(q, s)][j] for the lane's column j; one table block per 32 (16) columns of an
    // element, or a single block whose lanes cycle through an element's columns at the packed
    // pitch when several elements share a block
    for (int fam = 0; fam < 3; ++fam) {
        const int tm = fam_tm(fam), nrb = rblocks_of(P, fam);
        const bool packed = packed_columns(P, fam);
        const int tb = packed ? 1 : nrb, ng = groups_padded(P, fam), sl = fam_slots(fam);
        const size_t count = size_t(ng) * tb * 64 * sl;
        std::vector<double> v(count, 0.0);
        for (int g = 0; g < ng; ++g)
            for (int b = 0; b < tb; ++b)
                for (int l = 0; l < 64; ++l)
                    for (int sv = 0; sv < sl; ++sv) {
                        const int q = slot_point(fam, g, l, sv), r = slot_comp(sv);
                        const int j = packed ? (l % tm) % packed_pitch(P) : b * tm + l % tm;
                        if (q < nq && j < ns)
                            v[((size_t(g) * tb + b) * 64 + l) * sl + sv] = B[(size_t(q) * 4 + r) * ns + j];
                    }
        if (fam == MF_F64) {
            o.bcol[fam] = hb.put(v.data(), count * 8);
        } else {
            std::vector<float> f(v.begin(), v.end());
            o.bcol[fam] = hb.put(f.data(), count * 4);
        }
    }
    for (int prec = 0; prec < 5; ++prec) {
        const int fam = family_of(prec);
        const int ng = groups_padded(P, fam), nrb = rblocks_of(P, fam), sl = fam_slots(fam);
        const size_t count = size_t(ng) * nrb * 64 * sl;
        o.has_lo[prec] = false;
        if (prec == PREC_F64) {
            std::vector<double> v(count);
            for (int g = 0; g < ng; ++g)
                for (int rb = 0; rb < nrb; ++rb)
                    for (int l = 0; l < 64; ++l)
                        for (int k = 0; k < sl; ++k)
                            v[((size_t(g) * nrb + rb) * 64 + l) * sl + k] = row_value(B, P, fam, g, rb, l, k);
            o.row[prec][0] = hb.put(v.data(), count * 8);
        } else if (prec == PREC_F32) {
            std::vector<float> v(count);
            for (int g = 0; g < ng; ++g)
                for (int rb = 0; rb < nrb; ++rb)
                    for (int l = 0; l < 64; ++l)
                        for (int k = 0; k < sl; ++k)
                            v[((size_t(g) * nrb + rb) * 64 + l) * sl + k] = float(row_value(B, P, fam, g, rb, l, k));
            o.row[prec][0] = hb.put(v.data(), count * 4);
        } else {
            std::vector<uint16_t> hi(count), lo(count);
            for (int g = 0; g < ng; ++g)
                for (int rb = 0; rb < nrb; ++rb)
                    for (int l = 0; l < 64; ++l)
                        for (int k = 0; k < sl; ++k) {
                            const size_t idx = ((size_t(g) * nrb + rb) * 64 + l) * sl + k;
                            const double x = row_value(B, P, fam, g, rb, l, k);
                            if (prec == PREC_SPLIT_F16) {
                                const double y = x * double(F16_TABLE_SCALE);
                                hi[idx] = f16_bits(y);
                                lo[idx] = f16_bits(y - f16_value(hi[idx]));
                            } else {
                                hi[idx] = bf16_bits_rne(float(x));
                                lo[idx] = bf16_bits_rne(float(x - bf16_value(hi[idx])));
                            }
                        }
            o.row[prec][0] = hb.put(hi.data(), count * 2);
            if (prec != PREC_BF16) {
                o.row[prec][1] = hb.put(lo.data(), count * 2);
                o.has_lo[prec] = true;
            }
        }
    }
}

int build_tables(State &st)
{
    HostBlob hb;
    Offs offs[18];
    for (int p = 1; p <= 7; ++p) {
        HostDegreeTables t = make_degree_tables(p);
        const int n = t.n;
        std::vector<double> ld64(n * n * 2);
        std::vector<float> ld32(n * n * 2);
        for (int q = 0; q < n; ++q)
            for (int a = 0; a < n; ++a) {
                ld64[(q * n + a) * 2] = t.L[q * n + a];
                ld64[(q * n + a) * 2 + 1] = t.D[q * n + a];
                ld32[(q * n + a) * 2] = float(t.L[q * n + a]);
                ld32[(q * n + a) * 2 + 1] = float(t.D[q * n + a]);
            }
        Offs &o = offs[p];
        o.has_1d = true;
        o.xq = hb.put(t.xq.data(), n * 8);
        o.wq = hb.put(t.wq.data(), n * 8);
        o.ld64 = hb.put(ld64.data(), ld64.size() * 8);
        o.ld32 = hb.put(ld32.data(), ld32.size() * 4);
        o.c_bound = float(F16_C_TARGET / t.bmax);
        put_operand_tables(hb, o, p, reference_operand(t));
    }
    for (int p = 1; p <= 7; ++p) {
        HostPrismTables t;
        if (!make_prism_tables(p, t)) return FEM_ECONFIG;
        Offs &o = offs[PRISM_BASE + p];
        o.xq = hb.put(t.pts.data(), t.pts.size() * 8);  // [Nq][4]: xi1, xi2, zeta, weight
        o.phi64 = hb.put(t.phi.data(), t.phi.size() * 8);
        o.has_phi = true;
        o.c_bound = float(F16_C_TARGET / t.bmax);
        put_operand_tables(hb, o, PRISM_BASE + p, t.B);
    }
    void *d = nullptr;
    if (hipMalloc(&d, hb.bytes.size()) != hipSuccess) return FEM_ENOMEM;
    if (hipMemcpy(d, hb.bytes.data(), hb.bytes.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d);
        return FEM_EHIP;
    }
    st.blob = d;
    unsigned char *base = static_cast<unsigned char *>(d);
    for (int P = 1; P < 18; ++P) {
        if (P > 7 && P <= PRISM_BASE) continue;
        const Offs &o = offs[P];
        DegreeDev &dd = st.deg[P];
        dd.xq = reinterpret_cast<const double *>(base + o.xq);
        if (o.has_1d) {
            dd.wq = reinterpret_cast<const double *>(base + o.wq);
            dd.LD64 = reinterpret_cast<const double *>(base + o.ld64);
            dd.LD32 = reinterpret_cast<const float *>(base + o.ld32);
        }
        if (o.has_phi) dd.phi64 = reinterpret_cast<const double *>(base + o.phi64);
        dd.c_bound = o.c_bound;
        for (int fam = 0; fam < 3; ++fam) dd.bcol[fam] = base + o.bcol[fam];
        for (int prec = 0; prec < 5; ++prec) {
            dd.row[prec][0] = base + o.row[prec][0];
            dd.row[prec][1] = o.has_lo[prec] ? base + o.row[prec][1] : nullptr;
        }
    }
    return FEM_OK;
}

}  // namespace

namespace fem {
// p = 0 addresses the mixed-degree path: variant 0 is the single persistent launch over every
// degree, variant 1 one launch per degree. Keys MIXED_KEY + p (FEM_MIXED(p)) choose the tile
// degree p runs with inside the single launch (mixed_tile alternatives 0, 1).
constexpr int MIXED_SINGLE = 0, MIXED_PER_DEGREE = 1;
constexpr int MIXED_KEY = 20;
constexpr bool is_mixed_key(int p) { return p > MIXED_KEY && p <= MIXED_KEY + 7; }
static_assert(FEM_MIXED(1) == MIXED_KEY + 1, "one numbering of the mixed-launch tile keys");

int variant_count(int prec, int p)
{
    if (p == 0) return 2;
    if (is_mixed_key(p)) return prec >= PREC_F64 && prec <= PREC_SPLIT_F16 ? mixed_tile_count(p - MIXED_KEY, family_of(prec)) : 0;
    switch (prec) {
    case PREC_F64: return variants_f64(p);
    case PREC_F32: return variants_f32(p);
    case PREC_BF16: return variants_bf16(p);
    case PREC_SPLIT_BF16: return variants_split_bf16(p);
    case PREC_SPLIT_F16: return variants_split_f16(p);
    default: return 0;
    }
}

hipError_t dispatch_variant(int prec, int p, int v, const KArgs &a, hipStream_t s, int64_t cus)
{
    switch (prec) {
    case PREC_F64: return launch_f64(p, v, a, s, cus);
    case PREC_F32: return launch_f32(p, v, a, s, cus);
    case PREC_BF16: return launch_bf16(p, v, a, s, cus);
    case PREC_SPLIT_BF16: return launch_split_bf16(p, v, a, s, cus);
    case PREC_SPLIT_F16: return launch_split_f16(p, v, a, s, cus);
    default: return hipErrorInvalidValue;
    }
}

// The variant each (degree, precision, coefficient mode) launches: the measured default until
// fem_set_variant, fem_autotune or fem_load_tuning chooses another. Row 0: the mixed-degree
// strategy.
constexpr int NMODES = 3;
struct Choices {
    // [p] hexahedra (0: mixed strategy), [PRISM_BASE + p] prisms, [MIXED_KEY + p] the tile of
    // degree p inside the single mixed-degree launch
    int v[MIXED_KEY + 8][5][NMODES];
    Choices()
    {
        for (int prec = 0; prec < 5; ++prec)
            for (int mode = 0; mode < NMODES; ++mode) {
                v[0][prec][mode] = MIXED_PER_DEGREE;
                for (int p = 1; p <= 7; ++p) {
                    v[p][prec][mode] = default_variant(p, family_of(prec), mode);
                    v[PRISM_BASE + p][prec][mode] = default_variant(PRISM_BASE + p, family_of(prec), mode);
                    v[MIXED_KEY + p][prec][mode] = 0;
                }
            }
    }
};
Choices g_choice;

hipError_t dispatch(int prec, int mode, int p, const KArgs &a, hipStream_t s, int64_t cus)
{
    return dispatch_variant(prec, p, g_choice.v[p][prec][mode], a, s, cus);
}

hipError_t dispatch_mixed(int prec, const MixedKArgs &m, int64_t nel, hipStream_t s, int64_t cus)
{
    switch (prec) {
    case PREC_F64: return launch_mixed_f64(m, nel, s, cus);
    case PREC_F32: return launch_mixed_f32(m, nel, s, cus);
    case PREC_BF16: return launch_mixed_bf16(m, nel, s, cus);
    case PREC_SPLIT_BF16: return launch_mixed_split_bf16(m, nel, s, cus);
    case PREC_SPLIT_F16: return launch_mixed_split_f16(m, nel, s, cus);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace fem

namespace {

KArgs base_args(const fem_coeffs *c, const double *geom, void *out_A, void *out_b)
{
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.geom = geom;
    a.elem = c->elem;
    a.field = c->mode == FEM_COEF_FIELD ? c->field : nullptr;
    a.jac = c->jac;
    a.out_A = out_A;
    a.out_b = out_b;
    a.status = c->status;
    a.mode = c->mode;
    return a;
}

void set_degree(KArgs &a, int p, int prec)
{
    const DegreeDev &d = g_state.deg[p];
    a.xq = d.xq;
    a.wq = d.wq;
    a.LD64 = d.LD64;
    a.LD32 = d.LD32;
    a.phi64 = d.phi64;
    a.row_hi = d.row[prec][0];
    a.row_lo = d.row[prec][1];
    a.bcol = d.bcol[family_of(prec)];
    a.c_bound = d.c_bound;
    a.row_scale_inv = prec == PREC_SPLIT_F16 ? 1.0f / F16_TABLE_SCALE : 1.0f;
    a.a_stride = int64_t(ns_of(p)) * ns_of(p);
    a.b_stride = ns_of(p);
}

}  // namespace

extern "C" {

int fem_abi_version(void) { return FEM_ABI_VERSION; }

int fem_field_advance(double *field, const double *deltas, int32_t nsteps, int32_t *step,
                      void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (!field || !step || nsteps < 0 || (nsteps > 0 && !deltas)) return FEM_EINVAL;
    return field_advance(field, deltas, nsteps, step, (hipStream_t)stream) == hipSuccess ? FEM_OK
                                                                                         : FEM_EHIP;
}

int fem_gather_sample(int64_t nsel, const int32_t *sel, int32_t nrows, const int32_t *step,
                      int64_t nel, const int64_t *a_off, const int64_t *b_off, const void *A,
                      const void *b, int precision, void *out_A, int64_t cap_A, void *out_b,
                      int64_t cap_b, void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    if (nsel < 0 || nsel > INT32_MAX || nel < 0 || cap_A < 0 || cap_b < 0) return FEM_EINVAL;
    if (nsel == 0) return FEM_OK;
    if (!sel || nrows < 1 || !a_off || !A || !out_A) return FEM_EINVAL;
    if ((b != nullptr) != (out_b != nullptr) || (b && !b_off)) return FEM_EINVAL;
    const int32_t entry_bytes = precision == FEM_FP64 ? 8 : 4;
    return gather_sample(nsel, sel, nrows, step, nel, a_off, b_off, A, b, out_A, cap_A, out_b, cap_b,
                         entry_bytes, (hipStream_t)stream) == hipSuccess
               ? FEM_OK
               : FEM_EHIP;
}

int fem_reference_tables(int p, double *gauss_x, double *gauss_w, double *lobatto_x, double *L,
                         double *D)
{
    if (p < 1 || p > 7) return FEM_EDEGREE;
    const HostDegreeTables t = make_degree_tables(p);
    const int n = t.n;
    if (gauss_x) std::memcpy(gauss_x, t.xq.data(), n * sizeof(double));
    if (gauss_w) std::memcpy(gauss_w, t.wq.data(), n * sizeof(double));
    if (lobatto_x) lobatto_nodes(p, lobatto_x);
    if (L) std::memcpy(L, t.L.data(), n * n * sizeof(double));
    if (D) std::memcpy(D, t.D.data(), n * n * sizeof(double));
    return FEM_OK;
}

const char *fem_strerror(int status)
{
    switch (status) {
    case FEM_OK: return "success";
    case FEM_EINVAL: return "invalid argument";
    case FEM_EDEGREE: return "degree outside 1..7 (or p == 0 without a degree array)";
    case FEM_ENOTINIT: return "fem_init has not been called";
    case FEM_ENOMEM: return "device allocation failed";
    case FEM_EHIP: return "HIP runtime error";
    case FEM_ECONFIG: return "no kernel configuration for this request";
    case FEM_EWORKSPACE: return "workspace missing or too small";
    case FEM_ETOOBIG: return "more elements than the static scratch of fem_integrate_noalloc holds (FEM_NOALLOC_MAX_NEL)";
    default: return "unknown status";
    }
}

int fem_init(int device)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (g_state.blob && g_state.device == device) return FEM_OK;
    if (g_state.blob) return FEM_EINVAL;  // already initialised on another device
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FEM_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return FEM_EHIP;
    if (device < MAX_DEVICES && !g_scratch[device]) {
        void *ptr = nullptr;
        if (mixed_scratch_address(&ptr) != hipSuccess || !ptr) return FEM_EHIP;
        g_scratch[device] = ptr;
    }
    hipError_t e;
    if ((e = prepare_f64()) != hipSuccess || (e = prepare_f32()) != hipSuccess ||
        (e = prepare_bf16()) != hipSuccess || (e = prepare_split_bf16()) != hipSuccess ||
        (e = prepare_split_f16()) != hipSuccess || (e = mixed_prepare()) != hipSuccess ||
        (e = transpose_prepare()) != hipSuccess)
        return FEM_EHIP;
    const int rc = build_tables(g_state);
    if (rc != FEM_OK) return rc;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        g_cus = prop.multiProcessorCount;
    g_state.device = device;
    return FEM_OK;
}

int fem_finalize(void)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_state.blob) return FEM_ENOTINIT;
    (void)hipDeviceSynchronize();
    staged_release();
    (void)hipFree(g_state.blob);
    g_state = State();
    return FEM_OK;
}

int fem_jacobian_terms(int64_t nel, int p, const double *geom, const int8_t *degree,
                       const int64_t *b_off, double *jac, void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (nel < 0) return FEM_EINVAL;
    if (p < 0 || p > 7) return FEM_EDEGREE;
    if (p == 0 && !degree) return FEM_EDEGREE;
    if (p == 0 && !b_off) return FEM_EINVAL;
    if (nel == 0) return FEM_OK;
    if (!geom || !jac) return FEM_EINVAL;
    JacArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nel = nel;
    a.p = p;
    a.geom = geom;
    a.degree = degree;
    a.b_off = b_off;
    for (int pp = 1; pp <= 7; ++pp) a.xq[pp] = g_state.deg[pp].xq;
    a.out = jac;
    return jacobian_terms_launch(a, (hipStream_t)stream, g_cus) == hipSuccess ? FEM_OK : FEM_EHIP;
}

size_t fem_workspace_bytes(int64_t nel)
{
    return nel < 0 ? 0 : mixed_workspace_bytes(nel);
}

int fem_mixed_offsets(int64_t nel, const int8_t *degree, int64_t *a_off, int64_t *b_off,
                      void *workspace, size_t workspace_bytes, void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (nel < 0 || !a_off || !b_off || (nel > 0 && !degree)) return FEM_EINVAL;
    if (!workspace || workspace_bytes < mixed_workspace_bytes(nel)) return FEM_EWORKSPACE;
    return mixed_offsets(nel, degree, a_off, b_off, workspace, (hipStream_t)stream) == hipSuccess
               ? FEM_OK
               : FEM_EHIP;
}

}  // extern "C"

namespace {

// One element kind and degree P (hexahedron p or prism PRISM_BASE + p) over nel elements; the
// arguments are checked by the caller.
int integrate_uniform(int64_t nel, int P, const double *geom, const fem_coeffs *coeffs, void *out_A,
                      void *out_b, hipStream_t s)
{
    KArgs a = base_args(coeffs, geom, out_A, out_b);
    a.nel = nel;
    set_degree(a, P, coeffs->precision);
    if (coeffs->mode == FEM_COEF_ELASTIC) {
        // blocks (test component i, trial component k), one launch each, written with element
        // strides 9 Ns^2 and 3 Ns; the load vector of component i comes with block (i, i). Where
        // it pays, the blocks below the diagonal are the transposes of those above (major
        // symmetry of c_ijkl): copied by a separate kernel, or written by the upper block's
        // epilogue (at_base: the transposed block's offset, always > 0).
        const int64_t nsq = a.a_stride, ns = a.b_stride;
        // E_EPI needs the chosen tile's epilogue to write transposed blocks; otherwise the copy
        int em = elastic_mode(P, coeffs->precision);
        if (em == E_EPI && !trans_variant(coeffs->precision, P, g_choice.v[P][coeffs->precision][FEM_COEF_ELASTIC]))
            em = E_COPY;
        const bool sym = em != E_NINE;
        for (int i = 0; i < 3; ++i)
            for (int k = sym ? i : 0; k < 3; ++k) {
                KArgs ab = a;
                ab.comp_i = i;
                ab.comp_k = k;
                ab.a_base = (3 * i + k) * nsq;
                ab.at_base = (em == E_EPI && k > i) ? (3 * k + i) * nsq : 0;
                ab.a_stride = 9 * nsq;
                ab.b_base = i * ns;
                ab.b_stride = 3 * ns;
                ab.out_b = (i == k) ? out_b : nullptr;
                ab.status = (i == 0 && k == 0) ? coeffs->status : nullptr;
                if (dispatch(coeffs->precision, FEM_COEF_ELASTIC, P, ab, s, g_cus) != hipSuccess) return FEM_EHIP;
            }
        if (em == E_COPY && transpose_elastic_blocks(out_A, coeffs->precision == FEM_FP64, nel, (int)ns, s, g_cus) != hipSuccess)
            return FEM_EHIP;
        return FEM_OK;
    }
    return dispatch(coeffs->precision, coeffs->mode, P, a, s, g_cus) == hipSuccess ? FEM_OK : FEM_EHIP;
}

// fem_integrate with the mixed-degree workspace given explicitly (the caller's, or the static
// scratch of fem_integrate_noalloc).
int integrate_impl(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs, void *out_A,
                   void *out_b, void *stream, void *workspace, size_t workspace_bytes)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (nel < 0 || !coeffs) return FEM_EINVAL;
    if (coeffs->precision < FEM_FP64 || coeffs->precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    if (coeffs->mode != FEM_COEF_ELEMENT && coeffs->mode != FEM_COEF_FIELD &&
        coeffs->mode != FEM_COEF_ELASTIC)
        return FEM_EINVAL;
    if (p < 0 || p > 7) return FEM_EDEGREE;
    if (coeffs->mode == FEM_COEF_ELASTIC && p == 0) return FEM_EINVAL;
    if (p == 0 && !coeffs->degree) return FEM_EDEGREE;
    if (nel == 0) return FEM_OK;
    if (!out_A || !coeffs->elem || (!geom && !coeffs->jac)) return FEM_EINVAL;
    if (coeffs->mode == FEM_COEF_FIELD && (!coeffs->field || !geom)) return FEM_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    if (p > 0) return integrate_uniform(nel, p, geom, coeffs, out_A, out_b, s);
    KArgs a = base_args(coeffs, geom, out_A, out_b);
    // mixed degree: bucket on the device, then one launch per degree over its bucket
    if (!coeffs->a_off || ((out_b || coeffs->jac) && !coeffs->b_off)) return FEM_EINVAL;
    if (!workspace || workspace_bytes < mixed_workspace_bytes(nel)) return FEM_EWORKSPACE;
    MixedPlan plan;
    if (mixed_bucket(nel, coeffs->degree, workspace, s, &plan) != hipSuccess) return FEM_EHIP;
    a.a_off = coeffs->a_off;
    a.b_off = coeffs->b_off;
    MixedKArgs m;
    for (int pp = 1; pp <= 7; ++pp) {
        KArgs &ap = m.deg[pp - 1];
        ap = a;
        set_degree(ap, pp, coeffs->precision);
        ap.nel = nel;                  // upper bound; the bucket's count is read on the device
        ap.elist = plan.elist;
        ap.seg = plan.seg + 2 * pp;
        m.tile[pp - 1] = g_choice.v[MIXED_KEY + pp][coeffs->precision][coeffs->mode];
    }
    m.tile[7] = 0;
    if (g_choice.v[0][coeffs->precision][coeffs->mode] == MIXED_SINGLE)
        return dispatch_mixed(coeffs->precision, m, nel, s, g_cus) == hipSuccess ? FEM_OK : FEM_EHIP;
    for (int pp = 7; pp >= 1; --pp)  // heaviest degree first
        if (dispatch(coeffs->precision, coeffs->mode, pp, m.deg[pp - 1], s, g_cus) != hipSuccess) return FEM_EHIP;
    return FEM_OK;
}

}  // namespace

extern "C" {

int fem_integrate(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs, void *out_A,
                  void *out_b, void *stream)
{
    if (!coeffs) return FEM_EINVAL;
    return integrate_impl(nel, p, geom, coeffs, out_A, out_b, stream, coeffs->workspace,
                          coeffs->workspace_bytes);
}

int fem_integrate_prism(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                        void *out_A, void *out_b, void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (nel < 0 || !coeffs) return FEM_EINVAL;
    if (coeffs->precision < FEM_FP64 || coeffs->precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    if (coeffs->mode != FEM_COEF_ELEMENT && coeffs->mode != FEM_COEF_FIELD &&
        coeffs->mode != FEM_COEF_ELASTIC)
        return FEM_EINVAL;
    if (p < 1 || p > 7) return FEM_EDEGREE;
    if (coeffs->jac) return FEM_EINVAL;
    if (nel == 0) return FEM_OK;
    if (!out_A || !coeffs->elem || !geom) return FEM_EINVAL;
    if (coeffs->mode == FEM_COEF_FIELD && !coeffs->field) return FEM_EINVAL;
    return integrate_uniform(nel, PRISM_BASE + p, geom, coeffs, out_A, out_b, (hipStream_t)stream);
}

int fem_prism_reference_tables(int p, double *tri, double *B)
{
    if (p < 1 || p > 7) return FEM_EDEGREE;
    if (tri) {
        std::vector<double> x, y, w;
        if (!prism_triangle_rule(p, x, y, w)) return FEM_ECONFIG;
        for (size_t k = 0; k < x.size(); ++k) {
            tri[3 * k] = x[k];
            tri[3 * k + 1] = y[k];
            tri[3 * k + 2] = w[k];
        }
    }
    if (B) {
        HostPrismTables t;
        if (!make_prism_tables(p, t)) return FEM_ECONFIG;
        std::memcpy(B, t.B.data(), t.B.size() * sizeof(double));
    }
    return FEM_OK;
}

int fem_integrate_noalloc(int64_t nel, int p, const double *geom, const fem_coeffs *coeffs,
                          void *out_A, void *out_b, void *stream)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (!coeffs) return FEM_EINVAL;
    if (p == 0 && nel > FEM_NOALLOC_MAX_NEL) return FEM_ETOOBIG;
    const int dev = g_state.device;
    void *ws = (dev >= 0 && dev < MAX_DEVICES) ? g_scratch[dev] : nullptr;
    if (!ws) return FEM_ENOTINIT;
    return integrate_impl(nel, p, geom, coeffs, out_A, out_b, stream, ws,
                          mixed_workspace_bytes(FEM_NOALLOC_MAX_NEL));
}

}  // extern "C"

namespace {

// Seeded synthetic batch for fem_autotune: independent, mildly distorted unit cubes, with the
// records of the tuned coefficient mode (ELEMENT: an anisotropic SPD diffusion, a small
// convection and a reaction term; FIELD: a rotation and a load per element and a field
// descriptor of 7 fields x 5 modes; ELASTIC: Young modulus, Poisson ratio and body force), so
// that every variant runs the same arithmetic it runs on a real mesh.
struct TuneBatch {
    std::vector<double> geom, elem, field;
    int reclen = 14;
};
TuneBatch tune_batch(int64_t nel, int mode, bool prism)
{
    TuneBatch t;
    t.reclen = mode == FEM_COEF_ELEMENT ? 14 : (mode == FEM_COEF_FIELD ? 10 : 5);
    const int nv = prism ? 6 : 8;
    t.geom.resize(size_t(nel) * nv * 3);
    t.elem.assign(size_t(nel) * t.reclen, 0.0);
    uint64_t x = 0x9e3779b97f4a7c15ull;
    auto uni = [&x]() {  // xorshift64*, uniform in [-1, 1)
        x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
        return double((x * 0x2545f4914f6cdd1dull) >> 11) * 0x1.0p-52 - 1.0;
    };
    for (int64_t e = 0; e < nel; ++e) {
        for (int v = 0; v < nv; ++v)
            for (int d = 0; d < 3; ++d) {
                // hexahedron vertex v = v1 + 2 v2 + 4 v3; prism vertex v = t + 3 h (triangle vertex
                // t at (0,0), (1,0), (0,1), h the layer)
                const double ref = prism ? (d < 2 ? double(v % 3 == d + 1) : double(v / 3))
                                         : double((v >> d) & 1);
                t.geom[(e * nv + v) * 3 + d] = ref + 0.1 * uni();
            }
        double *r = &t.elem[e * t.reclen];
        if (mode == FEM_COEF_ELEMENT) {
            r[0] = 1.0 + 0.2 * uni(); r[4] = 1.0 + 0.2 * uni(); r[8] = 1.0 + 0.2 * uni();
            r[1] = r[3] = 0.1 * uni();
            r[9] = 0.3 * uni(); r[10] = 0.3 * uni(); r[11] = 0.3 * uni();
            r[12] = 1.0 + 0.5 * uni(); r[13] = uni();
        } else if (mode == FEM_COEF_FIELD) {
            // rotation about the third axis by a random angle, then the load
            const double a = 3.14159265358979 * uni(), c = std::cos(a), sn = std::sin(a);
            r[0] = c; r[1] = -sn; r[3] = sn; r[4] = c; r[8] = 1.0;
            r[9] = uni();
        } else {
            r[0] = 5.5 + 4.5 * uni(); r[1] = 0.3 + 0.1 * uni();
            r[2] = uni(); r[3] = uni(); r[4] = uni();
        }
    }
    if (mode == FEM_COEF_FIELD) {
        t.field.resize(175);
        for (int sm = 0; sm < 35; ++sm) {
            double *f = &t.field[sm * 5];
            f[0] = 0.2 * uni();
            for (int k = 1; k <= 3; ++k) f[k] = double(int(2.5 * (uni() + 1.0)) - 2);
            f[4] = 3.14159265358979 * (uni() + 1.0);
        }
    }
    return t;
}

const char *arch_name()
{
    static char name[64] = "";
    hipDeviceProp_t prop;
    if (!name[0] && hipGetDeviceProperties(&prop, g_state.device) == hipSuccess) {
        std::strncpy(name, prop.gcnArchName, sizeof(name) - 1);
        char *colon = std::strchr(name, ':');
        if (colon) *colon = '\0';
    }
    return name;
}

struct TuneEntry {
    int p, precision, mode, variant;
    double ms[FEM_MAX_VARIANTS];
    int count;
};

// Entries of a tuning file. Each entry sits on a line of its own:
//   {"p": 2, "precision": 4, "mode": 0, "variant": 0, "ms": [0.91, 1.02, 1.10]},
bool read_tuning(const char *path, std::string *arch, std::vector<TuneEntry> *out)
{
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char a[64];
        if (std::sscanf(line, " {\"arch\": \"%63[^\"]\"", a) == 1) *arch = a;
        TuneEntry t{};
        if (std::sscanf(line, " {\"p\": %d, \"precision\": %d, \"mode\": %d, \"variant\": %d", &t.p,
                        &t.precision, &t.mode, &t.variant) == 4) {
            const char *m = std::strstr(line, "\"ms\": [");
            if (m) {
                m += 7;
                int used = 0;
                while (t.count < FEM_MAX_VARIANTS && std::sscanf(m, " %lf%n", &t.ms[t.count], &used) == 1) {
                    ++t.count;
                    m += used;
                    while (*m == ' ' || *m == ',') ++m;
                }
            }
            out->push_back(t);
        }
    }
    std::fclose(f);
    return true;
}

bool write_tuning(const char *path, const std::string &arch, const std::vector<TuneEntry> &es)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"arch\": \"%s\", \"entries\": [\n", arch.c_str());
    for (size_t k = 0; k < es.size(); ++k) {
        const TuneEntry &t = es[k];
        std::fprintf(f, "  {\"p\": %d, \"precision\": %d, \"mode\": %d, \"variant\": %d, \"ms\": [", t.p,
                     t.precision, t.mode, t.variant);
        for (int v = 0; v < t.count; ++v) std::fprintf(f, "%s%.6g", v ? ", " : "", t.ms[v]);
        std::fprintf(f, "]}%s\n", k + 1 < es.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

// Keys of the variant tables: 0 (the mixed-degree strategy), 1..7 (hexahedra), FEM_PRISM(1..7),
// FEM_MIXED(1..7) (the tile of a degree inside the single mixed-degree launch).
bool valid_degree_key(int p)
{
    return (p >= 0 && p <= 7) || (p > PRISM_BASE && p <= PRISM_BASE + 7) || is_mixed_key(p);
}

}  // namespace

extern "C" {

int fem_variant_count(int p, int precision)
{
    if (!valid_degree_key(p)) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    return variant_count(precision, p);
}

int fem_get_variant(int p, int precision, int mode)
{
    if (!valid_degree_key(p)) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16 || mode < 0 || mode >= NMODES) return FEM_EINVAL;
    return g_choice.v[p][precision][mode];
}

int fem_set_variant(int p, int precision, int mode, int variant)
{
    if (!valid_degree_key(p)) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16 || mode < 0 || mode >= NMODES) return FEM_EINVAL;
    if (variant < 0 || variant >= variant_count(precision, p)) return FEM_ECONFIG;
    if (variant == trilinear_variant(p, family_of(precision)) && mode != FEM_COEF_ELEMENT) return FEM_ECONFIG;
    g_choice.v[p][precision][mode] = variant;
    return FEM_OK;
}

int fem_elastic_blocks(int p, int precision)
{
    if (!((p >= 1 && p <= 7) || (p > PRISM_BASE && p <= PRISM_BASE + 7))) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16) return FEM_EINVAL;
    return elastic_mode(p, precision) != E_NINE ? 6 : 9;
}

int fem_mixed_variant(int p, int precision, int mode)
{
    if (p < 1 || p > 7) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16 || mode < 0 || mode >= NMODES) return FEM_EINVAL;
    return mixed_tile(p, family_of(precision), g_choice.v[MIXED_KEY + p][precision][mode]);
}

int fem_autotune(int p, int precision, int mode, int64_t nel, const char *json_path, int *chosen,
                 double *times_ms)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (!valid_degree_key(p)) return FEM_EDEGREE;
    if (precision < FEM_FP64 || precision > FEM_SPLIT_FP16 || nel <= 0 || mode < 0 || mode >= NMODES)
        return FEM_EINVAL;
    if (mode == FEM_COEF_ELASTIC && (p == 0 || is_mixed_key(p))) return FEM_EINVAL;
    // p = 0: first the tile of each degree inside the single launch, each on a batch of that
    // degree alone of about the size its bucket has in the mix, then the strategy
    if (p == 0)
        for (int d = 7; d >= 1; --d) {
            const int64_t nd = std::max<int64_t>(1, nel * (8 - d) / 28);
            const int rc = fem_autotune(MIXED_KEY + d, precision, mode, nd, json_path, nullptr, nullptr);
            if (rc != FEM_OK) return rc;
        }
    const bool mixed_tile_key = is_mixed_key(p);
    const int dmix = mixed_tile_key ? p - MIXED_KEY : 0;  // the one degree of a tile key's batch
    const bool prism = is_prism(p) && !mixed_tile_key;
    const int nv = variant_count(precision, p);
    const size_t osz = precision == FEM_FP64 ? 8 : 4;
    const int64_t blocks = mode == FEM_COEF_ELASTIC ? 9 : 1, comps = mode == FEM_COEF_ELASTIC ? 3 : 1;
    const TuneBatch tb = tune_batch(nel, mode, prism);
    // p = 0: degrees 1..7 with weights 8 - p, interleaved; offsets by an exclusive scan
    std::vector<int8_t> deg;
    std::vector<int64_t> a_off(1, 0), b_off(1, 0);
    if (p == 0) {
        deg.resize(nel);
        uint64_t x = 0x2545f4914f6cdd1dull;
        for (int64_t e = 0; e < nel; ++e) {
            x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
            int r = int(((x * 0x9e3779b97f4a7c15ull) >> 33) % 28), d = 1;
            while (r >= 8 - d) { r -= 8 - d; ++d; }
            deg[e] = int8_t(d);
            const int64_t ns = ns_of(d);
            a_off.push_back(a_off.back() + ns * ns);
            b_off.push_back(b_off.back() + ns);
        }
    } else if (mixed_tile_key) {
        deg.assign(size_t(nel), int8_t(dmix));
        const int64_t ns = ns_of(dmix);
        for (int64_t e = 0; e < nel; ++e) {
            a_off.push_back(a_off.back() + ns * ns);
            b_off.push_back(b_off.back() + ns);
        }
    } else {
        a_off.push_back(nel * blocks * int64_t(ns_of(p)) * ns_of(p));
        b_off.push_back(nel * comps * int64_t(ns_of(p)));
    }
    const bool via_mixed = p == 0 || mixed_tile_key;  // the call goes through the mixed-degree path
    void *d_geom = nullptr, *d_elem = nullptr, *d_field = nullptr, *d_A = nullptr, *d_b = nullptr;
    void *d_deg = nullptr, *d_aoff = nullptr, *d_boff = nullptr, *d_ws = nullptr;
    const size_t ws_bytes = via_mixed ? mixed_workspace_bytes(nel) : 0;
    hipStream_t s = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = FEM_OK;
    double best_ms = 0.0;
    int best = 0;
    TuneEntry entry{p, precision, mode, 0, {}, nv};
    auto fail = [&](int code) { if (rc == FEM_OK) rc = code; };
    if (hipMalloc(&d_geom, tb.geom.size() * 8) != hipSuccess ||
        hipMalloc(&d_elem, tb.elem.size() * 8) != hipSuccess ||
        hipMalloc(&d_A, size_t(a_off.back()) * osz) != hipSuccess ||
        hipMalloc(&d_b, size_t(b_off.back()) * osz) != hipSuccess)
        fail(FEM_ENOMEM);
    if (rc == FEM_OK && !tb.field.empty() && hipMalloc(&d_field, tb.field.size() * 8) != hipSuccess)
        fail(FEM_ENOMEM);
    if (rc == FEM_OK && via_mixed &&
        (hipMalloc(&d_deg, nel) != hipSuccess || hipMalloc(&d_aoff, a_off.size() * 8) != hipSuccess ||
         hipMalloc(&d_boff, b_off.size() * 8) != hipSuccess || hipMalloc(&d_ws, ws_bytes) != hipSuccess))
        fail(FEM_ENOMEM);
    if (rc == FEM_OK && (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&ev[0]) != hipSuccess ||
                         hipEventCreate(&ev[1]) != hipSuccess))
        fail(FEM_EHIP);
    if (rc == FEM_OK &&
        (hipMemcpy(d_geom, tb.geom.data(), tb.geom.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(d_elem, tb.elem.data(), tb.elem.size() * 8, hipMemcpyHostToDevice) != hipSuccess))
        fail(FEM_EHIP);
    if (rc == FEM_OK && d_field &&
        hipMemcpy(d_field, tb.field.data(), tb.field.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
        fail(FEM_EHIP);
    if (rc == FEM_OK && via_mixed &&
        (hipMemcpy(d_deg, deg.data(), nel, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(d_aoff, a_off.data(), a_off.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
         hipMemcpy(d_boff, b_off.data(), b_off.size() * 8, hipMemcpyHostToDevice) != hipSuccess))
        fail(FEM_EHIP);
    fem_coeffs c;
    std::memset(&c, 0, sizeof(c));
    c.precision = precision;
    c.mode = mode;
    c.elem = static_cast<const double *>(d_elem);
    c.field = static_cast<const double *>(d_field);
    c.degree = static_cast<const int8_t *>(d_deg);
    c.a_off = static_cast<const int64_t *>(d_aoff);
    c.b_off = static_cast<const int64_t *>(d_boff);
    c.workspace = d_ws;
    c.workspace_bytes = ws_bytes;
    const int saved = g_choice.v[p][precision][mode];
    const int saved_strategy = g_choice.v[0][precision][mode];
    // each variant is timed through the whole call (every block of an elasticity call, the
    // bucketing of a mixed-degree call); a tile key's through the single mixed-degree launch
    auto run = [&](int v) -> bool {
        g_choice.v[p][precision][mode] = v;
        if (mixed_tile_key) g_choice.v[0][precision][mode] = MIXED_SINGLE;
        if (prism)
            return fem_integrate_prism(nel, deg_of(p), static_cast<const double *>(d_geom), &c, d_A, d_b, s) == FEM_OK;
        return fem_integrate(nel, via_mixed ? 0 : p, static_cast<const double *>(d_geom), &c, d_A, d_b, s) == FEM_OK;
    };
    constexpr int REPS = 5;
    bool any = false;
    for (int v = 0; v < nv && rc == FEM_OK; ++v) {
        if (v == trilinear_variant(p, family_of(precision)) && mode != FEM_COEF_ELEMENT) {
            entry.ms[v] = -1.0;  // ELEMENT mode only
            if (times_ms) times_ms[v] = -1.0;
            continue;
        }
        if (!run(v)) { fail(FEM_EHIP); break; }
        (void)hipEventRecord(ev[0], s);
        for (int r = 0; r < REPS; ++r)
            if (!run(v)) fail(FEM_EHIP);
        (void)hipEventRecord(ev[1], s);
        float ms = 0.0f;
        if (hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess)
            fail(FEM_EHIP);
        entry.ms[v] = double(ms) / REPS;
        if (times_ms) times_ms[v] = entry.ms[v];
        if (!any || entry.ms[v] < best_ms) { best_ms = entry.ms[v]; best = v; }
        any = true;
    }
    g_choice.v[p][precision][mode] = saved;
    g_choice.v[0][precision][mode] = saved_strategy;
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    if (s) (void)hipStreamDestroy(s);
    for (void *ptr : {d_geom, d_elem, d_field, d_A, d_b, d_deg, d_aoff, d_boff, d_ws}) (void)hipFree(ptr);
    if (rc != FEM_OK) return rc;
    g_choice.v[p][precision][mode] = best;
    entry.variant = best;
    if (chosen) *chosen = best;
    if (json_path) {
        std::string arch;
        std::vector<TuneEntry> es, keep;
        read_tuning(json_path, &arch, &es);
        for (const TuneEntry &t : es)
            if (!(t.p == p && t.precision == precision && t.mode == mode)) keep.push_back(t);
        keep.push_back(entry);
        if (!write_tuning(json_path, arch_name(), keep)) return FEM_EINVAL;
    }
    return FEM_OK;
}

int fem_load_tuning(const char *json_path, int *applied)
{
    if (!g_state.blob) return FEM_ENOTINIT;
    if (!json_path) return FEM_EINVAL;
    std::string arch;
    std::vector<TuneEntry> es;
    if (!read_tuning(json_path, &arch, &es)) return FEM_EINVAL;
    if (arch != arch_name()) return FEM_ECONFIG;
    int n = 0;
    for (const TuneEntry &t : es)
        if (fem_set_variant(t.p, t.precision, t.mode, t.variant) == FEM_OK) ++n;
    if (applied) *applied = n;
    return FEM_OK;
}

}  // extern "C"
