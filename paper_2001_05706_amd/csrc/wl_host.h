// wl_host.h -- host-side runtime of the library: errors, gauge handles,
// execution sets (systems x right-hand sides with device-resident tables),
// fields, the launch autotuner and the kernel timer.
#pragma once

#include <complex>
#include <cstdlib>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/wilson.h"
#include "wl_kernels.h"

namespace wl {

// ------------------------------------------------------------------ errors

wl_status set_error(wl_status s, const char *fmt, ...);
void clear_error();

#define WL_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return ::wl::set_error(WL_ERR_HIP, "%s: %s (%s:%d)", #call,       \
                                                     hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

#define WL_TRY(expr)                      \
    do {                                  \
        wl_status s_ = (expr);            \
        if (s_ != WL_OK) return s_;       \
    } while (0)

// true if [p, p + bytes) lies inside one device allocation
bool device_range_ok(const void *p, size_t bytes);

// ------------------------------------------------------------------ precision helpers

int spinor_site_bytes(int prec);  // bytes per site of a packed vector (incl. norm)
int chunk_bytes(int prec);
int nchunks(int prec);
bool prec_recon_ok(int prec, int recon);
int link_bytes(int prec, int recon);
constexpr int kStrideAlign = 64;
// Chunk-row stride of a vector: Vh rounded up to a whole number of waves, made
// an odd multiple of 64 sites.  Rows of a field (and the vectors of a set) then
// start an odd multiple of 1 KiB apart instead of a large power of two apart,
// so the rows a wave streams at once do not all fall into the same cache sets.
inline int padded(int vh)
{
    int n = (vh + kStrideAlign - 1) / kStrideAlign;
    if ((n & 1) == 0) ++n;
    return n * kStrideAlign;
}

}  // namespace wl

// ------------------------------------------------------------------ gauge handle

struct wl_gauge_s {
    wl::SysDesc geom;          // gauge pointer unset
    int device = 0;
    double *U = nullptr;       // canonical FP64 copy (device)
    void *packed[4][2] = {};   // [prec][recon == 12]
    // the stream each packed copy was built on and an event recorded behind the
    // packing kernel: a call on another stream waits for it before reading
    hipStream_t packed_on[4][2] = {};
    hipEvent_t packed_ev[4][2] = {};
    // clover term A and A^{-1} per value of kappa * c_sw, FP64 [0], FP32 [1], FP16 [2]
    struct Clover {
        double kc;
        void *A[3];
        void *Ainv[3];
        hipStream_t built_on;
        hipEvent_t built_ev;
    };
    std::vector<Clover> clovers;
    ~wl_gauge_s();
};

namespace wl {

wl_status gauge_packed(wl_gauge g, int prec, int recon, hipStream_t s, const void **out);
// packed clover term A and A^{-1} for kappa * c_sw = kc in the storage a hop of
// precision prec reads (FP64, FP32, and FP16 for FP16/BF16), built on first use
wl_status gauge_clover(wl_gauge g, double kc, int prec, hipStream_t s, const void **A, const void **Ainv);

// ------------------------------------------------------------------ execution sets

struct Field {
    void *p = nullptr;
    float *n = nullptr;  // FP16/BF16 norms
    int prec = -1;
};

struct Layout {
    int B = 0;
    int nblocks = 0;
    int npslots = 0;
    VecDesc *d_vec = nullptr;
    BlkMap *d_map = nullptr;
};

struct SysEntry {
    wl_gauge g;
    int nrhs;
    double kappa;
    double csw = 0.0;  // clover coefficient; 0: Wilson operator
};

// ExecSet::layout keys at and above kPairLayout denote pair layouts, at and
// above kPencilLayout pencil layouts
constexpr int kPairLayout = 1 << 16;
constexpr int kPencilLayout = 1 << 17;

// A set of systems (each a gauge handle with nrhs right-hand sides) whose
// vectors share every field and every launch.
class ExecSet {
public:
    ExecSet(const std::vector<SysEntry> &systems);
    ~ExecSet();
    wl_status init();

    std::vector<SysEntry> systems;
    bool has_clover = false;   // some system carries a clover term
    std::vector<VecDesc> vec;  // nblk / pslot0 filled per layout
    int nvec = 0;
    size_t total_sites = 0;    // sum of strides over vectors

    // The set's fields at precision prec are large against the 256 MB
    // last-level cache: eight of them (about what a solver iteration touches
    // besides the links) exceed it.  The iteration kernels then read and write
    // fields non-temporally, which keeps the links in that cache for the hops
    // (in FP32 and FP64 the update kernels store the field the next hop
    // reads -- p, r or s -- plainly).
    // WL_STREAM_FIELDS=0 or 1 overrides the choice (tests of both forms).
    bool stream_fields(int prec) const
    {
        const char *env = getenv("WL_STREAM_FIELDS");
        if (env && (env[0] == '0' || env[0] == '1')) return env[0] == '1';
        const double site = (double)nchunks(prec) * chunk_bytes(prec) + (prec == P_F16 || prec == P_BF16 ? 4 : 0);
        return 8.0 * (double)total_sites * site > 256.0 * 1024 * 1024;
    }

    // device tables: prec < 0 geometry only; recon 0: no links (geometry and clover term)
    wl_status sys_table(int prec, int recon, hipStream_t s, const SysDesc **out);
    // B > 0: blocks of B sites of one vector; B < 0: blocks of -B vectors on 64
    // sites; B >= kPairLayout: blocks of B - kPairLayout sites of two vectors;
    // B >= kPencilLayout: blocks of one vector on the same 64 positions of
    // B - kPencilLayout consecutive time slices (every system's slices must
    // hold a multiple of 64 sites and its time extent be a multiple of the
    // slice count; WL_ERR_ARG otherwise)
    // col: z-planes per column of the block order (see the definition)
    wl_status layout(int B, const Layout **out, int col = 4);
    int32_t *d_active = nullptr;
    std::vector<int32_t> h_active;
    // copy h_active to d_active, ordered on the stream (no host synchronisation);
    // skipped when the same mask was the last one enqueued on the same stream
    wl_status upload_active(hipStream_t s);
    static constexpr int kMaskRing = 16;
    int32_t *h_masks = nullptr;  // pinned staging slots of the mask uploads
    hipEvent_t mask_ev[kMaskRing] = {};
    int mask_next = 0;
    std::vector<int32_t> up_active;  // the mask last enqueued for d_active
    hipStream_t up_stream = nullptr; // and its stream
    bool up_valid = false;
    hipEvent_t rr_ev = nullptr;      // marks a readback the host waits for while later work runs

    // reduction state (per vector unless noted)
    double *partials = nullptr;  // max slots over layouts (B = 64), 3 values each
    double *sc = nullptr;        // scalar arena, see SC_* below
    int32_t *bad = nullptr;      // at the end of the hist allocation
    double *hist = nullptr;      // residual history: [kHist][nvec], then bad
    double *hist_partials = nullptr;  // deferred block partials of the history: [kHist][max_pslots]
    double *h_pinned = nullptr;  // pinned host mirror of hist, scalars and flags
    static constexpr int kHist = 64;

    static constexpr int SC_N = SC_COUNT;  // scalar slots per vector (ScSlot)
    double *scal(int which) { return sc + (size_t)which * nvec; }

    // fields by name, allocated on first use
    wl_status field(const std::string &name, int prec, Field *out);
    // device scratch by name, grown on demand (contents not kept across growth)
    wl_status buffer(const std::string &name, size_t bytes, void **out);
    std::map<std::string, std::pair<void *, size_t>> bufs;

    std::map<std::pair<int, int>, SysDesc *> d_sys;
    std::map<std::pair<int, int>, Layout> layouts;  // by (block shape, column height)
    std::map<std::string, Field> fields;
    std::map<std::vector<double>, double *> coefs;
    std::map<std::string, hipGraphExec_t> graphs;  // captured iteration chunks
    int max_pslots = 0;
};

// Find or build the cached set for these systems (fields persist between calls).
wl_status get_set(const std::vector<SysEntry> &systems, ExecSet **out);
void drop_sets_of(wl_gauge g);

// ------------------------------------------------------------------ launches on a set

struct Epi {
    int nx = 0;
    int g5 = 0;
    int clov = 0;  // EPI_CLOV_* bits (act only on systems with a clover term)
    const double *coef = nullptr;  // device [nsys][5]
    Field X[4];
};

RedSpec no_red();
RedSpec red_spec(ExecSet &S, int kind, double *dst, int nv = 1, int mode = RM_NORM);

// out_p = epilogue(hop(in_{1-p})) on every active vector of the set
wl_status hop(ExecSet &S, int prec, int recon, bool dag, int out_parity, const Field &out, const Field &in,
              const Epi &e, const RedSpec &red, hipStream_t s, bool use_active = true);
// out_p = epi_p(hop(in_{1-p})) for both parities p (no reduction), in one launch
// when the set is a single vector
wl_status hop2(ExecSet &S, int prec, int recon, bool dag, const Field out[2], const Field in[2], const Epi e[2],
               hipStream_t s, bool use_active = true);
// bcast: bit j marks field j as a single vector shared by every vector of the set
wl_status blas(ExecSet &S, int op, int prec, const Field *f, int nf, const double *s0, const RedSpec &red,
               hipStream_t s, bool use_active = true, int parity = 0, int bcast = 0);
wl_status convert(ExecSet &S, const Field &dst, const Field &src, hipStream_t s, bool use_active = true);
// canonical <-> packed for one parity; canon[i] is the canonical field array of system i
wl_status pack(ExecSet &S, const double *const *canon, int parity, const Field &f, hipStream_t s);
wl_status unpack(ExecSet &S, double *const *canon, int parity, const Field &f, hipStream_t s);
wl_status zero_canon(ExecSet &S, double *const *canon, int parity, hipStream_t s);

// sum the deferred |r|^2 partials of the last k iterations into hist rows 0..k-1
wl_status hist_finalize(ExecSet &S, int k, hipStream_t s);

// device coefficient tables [nsys][5], cached by content
wl_status coef_table(ExecSet &S, const std::vector<double> &c, const double **out);

// ------------------------------------------------------------------ sign function (sign.hip)

// Chebyshev plan of eps(H_W) ~= s^{-1/2} H_W p(H_W^2 / s) for a single-system
// set: device coefficient rows [0] H_W, [1 .. N-1] Clenshaw steps, [N] final p v.
struct SignPlan {
    int N = 0;       // degree + 1
    double m = 0;    // 4 - rho
    double rs = 0;   // s^{-1/2}
    const double *tab = nullptr;
};
wl_status sign_plan(ExecSet &S, double rho, int degree, double lo, double hi, double scale, SignPlan *P);
// y = p(H_W^2 / s) v on both parities of every active vector; y aliases scratch
// fields of the set that the next sign_poly call in the same precision reuses
wl_status sign_poly(ExecSet &S, int prec, int recon, const SignPlan &P, const Field v[2], Field y[2], hipStream_t s);
// out_p = G5(a0 in_p + c hop(in)_p) on both parities with the coefficient row coef
wl_status apply_hw(ExecSet &S, int prec, int recon, const Field out[2], const Field in[2], const double *coef,
                   const RedSpec *red, hipStream_t s);
wl_status power_lmax(ExecSet &S, double rho, int recon, int iters, const Field u[2], double *lmax, hipStream_t s);
wl_status hw2_scale(wl_gauge U, double rho, const double *v0, hipStream_t s, double *scale);

// ------------------------------------------------------------------ low-mode deflation (eigs.hip)

// nev eigenpairs of H_W packed as the vectors of a single-system set
struct Deflation {
    int nev = 0;
    ExecSet *E = nullptr;
    std::vector<double> lam;  // eigenvalues of H_W
    Field f64[2], f32[2];     // packed eigenvectors per parity, FP64 and FP32
};
// pack nev canonical eigenvectors (device) and their eigenvalues (host); nev = 0: none
wl_status defl_load(wl_gauge U, double kappa, int nev, const double *evecs, const double *evals, hipStream_t s,
                    Deflation *D);
// c[i * nvec + v] = <xi_i, in_v> over both parities (host result)
wl_status defl_coeffs(ExecSet &S, const Deflation &D, int prec, const Field in[2], std::vector<std::complex<double>> &c,
                      hipStream_t s);
// y_v += sum_i z[i * nvec + v] (g5) xi_i over both parities
wl_status defl_axpy(ExecSet &S, const Deflation &D, int prec, const Field y[2], const std::vector<std::complex<double>> &z,
                    bool g5, hipStream_t s);

// ------------------------------------------------------------------ tuning and timing

int tuned_block(const std::string &key, const std::vector<int> &cands, hipStream_t s,
                const std::function<hipError_t(int)> &run);
bool capturing(hipStream_t s);
std::string hop_key(const ExecSet &S, int prec, int recon, bool dag);
std::vector<int> hop_candidates(int prec);
int cfg_make(int var, int block, int col);  // hop launch configuration: variant, block size, column height
int cfg_var(int c);
int cfg_block(int c);
int cfg_col(int c);

// Kernel timing of hop launches (eager launches only: a solver runs without
// graphs while timing is on).  Each timed launch carries start/end events that
// its dispatch records, and its blocks store steady-clock readings at their
// start and end, from which the kernel's own duration follows.
struct EventList {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> gbytes;
};
struct Prof {
    bool on = false;
    int prec = -1;  // storage precision of the hops timed (-1: all)
    int64_t launches = 0;
    double ms = 0.0;         // dispatch events
    double kernel_ms = 0.0;  // device steady clock: first block start to last block end
    double gbytes = 0.0;
    EventList pending;
    unsigned long long *d_stamps = nullptr;  // device block stamps of one launch
    std::vector<unsigned long long> h_stamps;
    size_t nstamps = 0;
    double clock_khz = 0.0;
};
Prof &prof();
void prof_collect();

// algorithmic bytes of one hop on all active vectors of the set
double hop_bytes(const ExecSet &S, int prec, int recon, bool use_active);
double blas_bytes(const ExecSet &S, int prec, int passes, bool use_active);
// algorithmic bytes of reading one packed clover field at every output site of the clover systems
double clover_bytes(const ExecSet &S, int prec, bool use_active);
extern thread_local double g_bytes_acc;  // running algorithmic-byte counter of the current call

}  // namespace wl
