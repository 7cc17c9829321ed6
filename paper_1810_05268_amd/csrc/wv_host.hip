// Host runtime and C ABI of libwv: validation, set-up tables, the Revolve schedule,
// and the executor that runs a schedule as a stream of kernel launches.
//
// Paper: Kukreja et al., "Combining checkpointing and data compression to
// accelerate adjoint-based optimization problems".  The executor follows the
// checkpointing runtime model of Sec. "Checkpointing performance model": the
// operator's working memory holds the current state; a store copies it into
// separate checkpoint memory, a restore copies it back (eq. (4)); with a
// tolerance the copies pass through the codec (eq. (6)) and the slot count grows
// by the compression ratio.
#include <cstdlib>
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "wv_internal.h"

using namespace wv;

namespace {

constexpr int ADVANCE = 1, STORE = 2, RESTORE = 3, FREE = 4, REVERSE = 5;

// ------------------------------------------------------------------ finite differences
// a_k = 2(-1)^(k+1)/k^2 * prod_{i=1..k} (K-k+i)/(K+i), a_0 = -2 sum a_k
// ((K!)^2 / ((K-k)!(K+k)!) written as a product of k ratios).
void fd_weights(int K, double *a)
{
    double s = 0.0;
    for (int k = 1; k <= K; ++k) {
        double r = 1.0;
        for (int i = 1; i <= k; ++i) r *= (double)(K - k + i) / (double)(K + i);
        const double v = 2.0 * r / ((double)k * (double)k);
        a[k] = (k & 1) ? v : -v;
        s += a[k];
    }
    a[0] = -2.0 * s;
}

// Stability limit: a mode with lam = c^2 dt^2 times its eigenvalue of -lap is stable for
// lam <= 4 under OT2 and for lam <= 12 under OT4 (which advances it with lam - lam^2/12).
double cfl_limit(int ndim, const double *h, int order, double vmax, int time_order = 2)
{
    if (ndim < 2 || ndim > 3 || order < 2 || order > 16 || (order & 1) || !(vmax > 0)) return -1.0;
    double a[kMaxK + 1];
    const int K = order / 2;
    fd_weights(K, a);
    double S = std::fabs(a[0]);
    for (int k = 1; k <= K; ++k) S += 2.0 * std::fabs(a[k]);
    double q = 0.0;
    for (int d = 0; d < ndim; ++d) {
        if (!(h[d] > 0)) return -1.0;
        q += S / (h[d] * h[d]);
    }
    return (time_order == 4 ? std::sqrt(12.0) : 2.0) / (vmax * std::sqrt(q));
}

// ------------------------------------------------------------------ schedule
constexpr long long kSat = (long long)1 << 62;

// C(c+r, c), saturating
long long binom(int c, long long r)
{
    if (r < 0 || c < 0) return 0;
    long long res = 1;
    for (long long i = 1; i <= r; ++i) {
        __int128 t = (__int128)res * (c + i);
        t /= i;
        if (t >= kSat) return kSat;
        res = (long long)t;
    }
    return res;
}

// min { r : beta(c, r) >= l }, stepping beta(c, r) = beta(c, r-1) (c+r) / r (exact)
int repetitions(long long l, int c)
{
    int r = 0;
    long long b = 1;
    while (b < l) {
        ++r;
        const __int128 t = (__int128)b * (c + r) / r;
        b = t >= kSat ? kSat : (long long)t;
    }
    return r;
}

long long forward_steps(long long nt, int M)
{
    const long long l = nt + 1;
    if (l <= 1) return 0;
    if (M <= 1) return l * (l - 1) / 2;
    const int r = repetitions(l, M);
    return r * l - binom(M + 1, r - 1);
}

struct Frame {
    int s;
    long long l;
    int c, slot;
    long long k;
    int nslot, phase;
};

// Write-minimal tie-break.  Every split takes a first advance from Griewank's optimal
// interval (so the forward-step count stays minimal); among those, the k that minimises
// the checkpoint writes of the whole recursion (smallest such k):
//   W(l, c) = min_{k in [lo, hi]} f(k),  f(k) = [l-k > 1] + W(l-k, c-1) + W(k, c),
//   W(1, c) = W(l, 1) = 0,
// where a right part of a single state stores nothing: that state is the one just
// reached and is reversed at once from the working state, so a checkpoint of it would
// never be read.  Where c >= l-1 every state fits and k = 1, W = l-2.  Where two
// repetitions suffice (beta(c, 2) >= l) the minimum is W = l-2-min(c, l-1-c).  Over the
// optimal interval f is convex (its differences never decrease), so the smallest
// minimiser is the first k whose forward difference is >= 0, found by bisection.  Both
// facts hold on every entry the full programme (a scan of the interval) was compared on;
// the schedules are checked against it.  The table holds the entries with
// beta(c, 2) < l (c < sqrt(2l)), column by column, for the slot counts asked for so far;
// it is kept per thread and reused by later schedules of the same length (the planner
// asks for many slot counts of one run).
struct WriteMin {
    long long L = 0;
    int C = 1;                  // columns 2..C are built
    std::vector<int32_t> W, K;  // [c * (L+1) + l], used where beta(c, 2) < l
    int32_t w(long long l, int c) const
    {
        if (l <= 2 || c <= 1) return 0;
        if (c >= l - 1) return (int32_t)(l - 2);
        if (binom(c, 2) >= l) return (int32_t)(l - 2 - std::min<long long>(c, l - 1 - c));
        return W[(size_t)c * (L + 1) + l];
    }
};

thread_local WriteMin g_wmin;

// Griewank's set of optimal first advances for a segment of l steps and c slots (c >= 2):
// the interval [max(beta(c,r-2), l-beta(c-1,r), 1), min(beta(c,r-1), l-beta(c-1,r-1), l-1)].
void optimal_interval(long long l, int c, long long &lo, long long &hi)
{
    const int r = repetitions(l, c);
    lo = std::max(std::max(binom(c, r - 2), l - binom(c - 1, r)), 1LL);
    hi = std::min(std::min(binom(c, r - 1), l - binom(c - 1, r - 1)), l - 1);
}

// the write-minimal first advance and the writes it leads to
long long best_split(const WriteMin &t, long long l, int c, int32_t *writes)
{
    long long lo, hi;
    optimal_interval(l, c, lo, hi);
    auto f = [&](long long k) { return (int32_t)(l - k > 1) + t.w(l - k, c - 1) + t.w(k, c); };
    while (lo < hi) {
        const long long mid = lo + (hi - lo) / 2;
        if (f(mid + 1) >= f(mid)) hi = mid;
        else lo = mid + 1;
    }
    if (writes) *writes = f(lo);
    return lo;
}

// columns the table needs for L states and up to M slots: those with an entry where
// beta(c, 2) < l
int write_min_columns(long long L, int M)
{
    int C = 1;
    while (C < M && binom(C + 1, 2) < L) ++C;
    return C;
}

// The table holds (C+1)(L+1) entries of each kind; a reversal that would need more is
// scheduled with the smallest optimal split instead (still minimal in forward steps).
constexpr long long kWriteMinEntries = 1LL << 26;

bool write_min_fits(long long L, int M)
{
    return (long long)(write_min_columns(L, M) + 1) * (L + 1) <= kWriteMinEntries;
}

// the table for schedules of L states with up to M slots
const WriteMin &write_min_table(long long L, int M)
{
    WriteMin &t = g_wmin;
    if (t.L != L) {
        t.L = L;
        t.C = 1;
        t.W.clear();
        t.K.clear();
        t.W.shrink_to_fit();
        t.K.shrink_to_fit();
    }
    const int C = write_min_columns(L, M);
    if (C <= t.C) return t;
    t.W.resize((size_t)(C + 1) * (L + 1), 0);
    t.K.resize((size_t)(C + 1) * (L + 1), 1);
    for (int c = t.C + 1; c <= C; ++c)
        for (long long l = binom(c, 2) + 1; l <= L; ++l) {   // beta(c, 2) < l (so c < l-1)
            int32_t wv = 0;
            const long long k = best_split(t, l, c, &wv);
            t.W[(size_t)c * (L + 1) + l] = wv;
            t.K[(size_t)c * (L + 1) + l] = (int32_t)k;
        }
    t.C = C;
    return t;
}

// The reversal of nt steps with M slots.  write_min: the write-minimal first advance,
// for slots of one size (exact copies), where every optimal split peaks at the same
// memory and fewer writes cost nothing (unless its table would exceed kWriteMinEntries).
// Otherwise the smallest optimal first advance, for compressed slots: their streams grow
// over the run (late states compress worst), and the smallest splits hold the earliest
// states, so more slots fit a budget.
void make_schedule(int nt, int M, bool write_min, std::vector<int32_t> &out)
{
    out.clear();
    const long long L = (long long)nt + 1;
    write_min = write_min && write_min_fits(L, M);
    // every segment of the recursion has c <= M, and c >= l-1 throughout when M >= L-1
    const WriteMin *tab = (write_min && M >= 2 && M < L - 1) ? &write_min_table(L, M) : nullptr;
    auto split = [&](long long l, int c) -> long long {
        if (c >= l - 1) return 1;
        if (!write_min) {
            long long lo, hi;
            optimal_interval(l, c, lo, hi);
            return lo;
        }
        if (binom(c, 2) < l) return tab->K[(size_t)c * (L + 1) + l];
        return best_split(*tab, l, c, nullptr);
    };
    int wm = 0, depth = 0;
    auto emit = [&](int op, long long a, long long b) {
        out.push_back(op);
        out.push_back((int32_t)a);
        out.push_back((int32_t)b);
    };
    auto need = [&](int s, int slot) {
        if (wm != s) {
            emit(RESTORE, s, slot);
            wm = s;
        }
    };
    std::vector<Frame> st;
    st.push_back({0, (long long)nt + 1, M, 0, 0, 0, 0});
    while (!st.empty()) {
        const Frame f = st.back();
        st.pop_back();
        if (f.phase == 1) {           // right part done: release its checkpoint, then the left part
            emit(FREE, f.s + f.k, f.nslot);
            --depth;
            st.push_back({f.s, f.k, f.c, f.slot, 0, 0, 0});
            continue;
        }
        if (f.l == 1) {
            if (f.s > 0) {
                need(f.s, f.slot);
                emit(REVERSE, f.s, 0);
            }
            continue;
        }
        if (f.c == 1) {
            for (long long i = f.l - 1; i >= 0; --i) {
                if (f.s + i == 0) break;
                need(f.s, f.slot);
                if (i > 0) {
                    emit(ADVANCE, f.s, f.s + i);
                    wm = (int)(f.s + i);
                }
                emit(REVERSE, f.s + i, 0);
            }
            continue;
        }
        const long long k = split(f.l, f.c);
        need(f.s, f.slot);
        emit(ADVANCE, f.s, f.s + k);
        wm = (int)(f.s + k);
        if (write_min && f.l - k == 1) {   // reversed at once from the working state: no checkpoint
            emit(REVERSE, f.s + k, 0);
            st.push_back({f.s, k, f.c, f.slot, 0, 0, 0});
            continue;
        }
        ++depth;
        emit(STORE, f.s + k, depth);
        st.push_back({f.s, f.l, f.c, f.slot, k, depth, 1});
        st.push_back({(int)(f.s + k), f.l - k, f.c - 1, depth, 0, 0, 0});
    }
}

// ------------------------------------------------------------------ set-up
thread_local char g_detail[256] = "";

int hip_fail(hipError_t e, const char *what, int line)
{
    std::snprintf(g_detail, sizeof(g_detail), "%s (line %d): %s", what, line, hipGetErrorString(e));
    return WV_EHIP;
}

#define HIPCHK(x)                                            \
    do {                                                     \
        const hipError_t e_ = (x);                           \
        if (e_ != hipSuccess) return hip_fail(e_, #x, __LINE__); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    size_t bk, U0, U1, L0, L1, W, Z, UB, DB, V, VU, CR;
    size_t src_tab, rec_tab, tab_bytes;
    size_t res, dsim, partials, enc, offs, sizes, arena;
    size_t total;
    size_t arena_bytes;
    long long nchunks_max;
    int offs_n;
};

constexpr size_t kBk = 4096;
// bookkeeping words inside bk
constexpr size_t kErr = 0, kMisfit = 128, kStats = 192, kZero = 256, kProbeNext = 264, kScal = 320;
constexpr int kParts = 1024;

struct Setup {
    Grid g;
    long long P = 0;        // grid points (the caller's dense arrays)
    long long Pf = 0;       // elements of one solver field array (rows pitched, see Grid)
    int ndim = 0, N[3] = {1, 1, 1};
    int src_nc = 4, rec_nc = 4;   // corners per source / receiver in the gather tables
    // host tables, packed
    std::vector<int> src_gidx, rec_gidx, src_pts, src_start, src_col, rec_pts, rec_start, rec_col;
    std::vector<float> src_gwt, rec_gwt, src_swt, rec_swt;
};

// A reverse step k reads only u^k.  The second level u^{k-1} of a checkpoint is
// needed only if the schedule advances from a restore of it: flag those STORE actions
// (by action index) so that only they write, and their restores only then decode, it.
std::vector<char> second_level_needed(const std::vector<int32_t> &acts, int M)
{
    const size_t nact = acts.size() / 3;
    std::vector<char> need2(nact, 0);
    std::vector<long> holder((size_t)M + 2, -1);   // slot -> index of the STORE that filled it
    for (size_t i = 0; i < nact; ++i) {
        const int op = acts[3 * i], b = acts[3 * i + 2];
        if (op == STORE && b >= 0 && b <= M) holder[b] = (long)i;
        if (op == RESTORE && b > 0 && b <= M && holder[b] >= 0) {
            size_t j = i + 1;
            while (j < nact && acts[3 * j] == FREE) ++j;
            if (j >= nact || acts[3 * j] != REVERSE) need2[holder[b]] = 1;
        }
    }
    return need2;
}

// What the executor does for a schedule, without a device: the counts that price it.
struct DryRun {
    long advances = 0, stores = 0, fields = 0, restores = 0, decodes = 0, reverses = 0;
};

DryRun dry_run(const std::vector<int32_t> &acts, int M, bool compressed)
{
    DryRun r;
    const std::vector<char> need2 = second_level_needed(acts, M);
    std::vector<char> slot2((size_t)M + 2, 0);
    int hot_slot = -1, hot_k = -1;
    bool hot_db = false, pending = false;
    for (size_t i = 0; i < acts.size() / 3; ++i) {
        const int op = acts[3 * i], a = acts[3 * i + 1], b = acts[3 * i + 2];
        switch (op) {
        case ADVANCE:
            if (pending) {
                if (compressed && !hot_db) {
                    ++r.decodes;
                    hot_db = true;
                }
                pending = false;
            }
            r.advances += b - a;
            break;
        case STORE:
            slot2[b] = need2[i];
            r.fields += need2[i] ? 2 : 1;
            ++r.stores;
            if (hot_slot == b) hot_slot = -1;
            break;
        case RESTORE:
            pending = false;
            if (b > 0) {
                if (compressed && (hot_slot != b || hot_k != a)) {
                    ++r.decodes;
                    hot_slot = b;
                    hot_k = a;
                    hot_db = false;
                }
                pending = slot2[b] != 0;
            }
            ++r.restores;
            break;
        case REVERSE:
            ++r.reverses;
            break;
        default:
            break;
        }
    }
    return r;
}

// Checkpoint slots M for a budget: x_0 (the zero state, no memory) plus as many stored
// states as fit; uncompressed slots hold S bytes, a compressed slot S / F plus the
// 256-byte alignment of its two streams (F is a ratio of whole streams, prefixes
// included).  M = 1 (a budget below one checkpoint) is recomputation from x_0 alone.
int plan_slots(int nt, size_t mem_budget, size_t S, bool compressed, double F)
{
    size_t slot_bytes = compressed ? (size_t)((double)S / F) + 512 : S;
    if (slot_bytes < 1) slot_bytes = 1;
    const size_t nslots = mem_budget / slot_bytes;
    return std::max(1, (int)std::min<size_t>((size_t)nt, nslots + 1));
}

// ------------------------------------------------- compressibility profile planning
// A profile is kProfile stream sizes (bytes) of one compressed field: prof[0] at k = 0
// (the empty field) and prof[j] at k_j = ceil(j N / (kProfile - 1)), j >= 1; 0 = unknown.
constexpr int kProfile = WV_PROFILE;

long long profile_step(int N, int j) { return (j * (long long)N + kProfile - 2) / (kProfile - 1); }

// whether a run that stores states 1..N-1 must store state k for the compressibility
// profile: a sample step, or the nearest stored state to one (N - 1 for k = N)
bool profile_sample(int N, long long k)
{
    for (int j = 1; j < kProfile; ++j)
        if (std::min<long long>(std::max<long long>(profile_step(N, j), 1), N - 1) == k) return true;
    return false;
}

void profile_from_sizes(const std::vector<uint64_t> &sz, int N, double empty_bytes, double *prof)
{
    prof[0] = empty_bytes;
    for (int j = 1; j < kProfile; ++j) {
        const long long kj = std::min<long long>(std::max<long long>(profile_step(N, j), 1), N);
        prof[j] = 0.0;
        for (long long dk = 0; dk <= N; ++dk) {   // nearest state that was stored
            if (kj - dk >= 1 && sz[kj - dk]) { prof[j] = (double)sz[kj - dk]; break; }
            if (kj + dk <= N && sz[kj + dk]) { prof[j] = (double)sz[kj + dk]; break; }
        }
    }
}

bool profile_valid(const double *prof)
{
    for (int j = 0; j < kProfile; ++j)
        if (!(prof[j] > 0)) return false;
    return true;
}

// stream bytes of u^k, linear between the samples
double profile_size(const double *prof, int N, long long k)
{
    for (int j = 1; j < kProfile; ++j) {
        const long long k0 = j == 1 ? 0 : profile_step(N, j - 1), k1 = profile_step(N, j);
        if (k <= k1 || j == kProfile - 1) {
            const double t = k1 > k0 ? (double)(k - k0) / (double)(k1 - k0) : 1.0;
            return prof[j - 1] + std::min(1.0, std::max(0.0, t)) * (prof[j] - prof[j - 1]);
        }
    }
    return prof[kProfile - 1];
}

// Peak bytes of the checkpoint arena for M slots: every stored state takes its stream
// (twice for the checkpoints that keep both levels, the increment taken as large as u),
// each rounded up to 256 bytes; slots are freed last-in first-out.
double simulate_peak(int N, int M, const double *prof)
{
    std::vector<int32_t> acts;
    make_schedule(N, M, false, acts);
    const std::vector<char> need2 = second_level_needed(acts, M);
    std::vector<double> held((size_t)M + 2, 0.0);
    double live = 0.0, peak = 0.0;
    for (size_t i = 0; i < acts.size() / 3; ++i) {
        const int op = acts[3 * i], a = acts[3 * i + 1], b = acts[3 * i + 2];
        if (op == STORE) {
            const double one = std::ceil(profile_size(prof, N, a) / 256.0) * 256.0;
            held[b] = need2[i] ? 2.0 * one : one;
            live += held[b];
            peak = std::max(peak, live);
        } else if (op == FREE) {
            live -= held[b];
            held[b] = 0.0;
        }
    }
    return peak;
}

// Largest M whose simulated peak fits mem_budget (3 % kept for the estimate's error).
int plan_slots_profile(int N, size_t mem_budget, const double *prof)
{
    const double lim = 0.97 * (double)mem_budget;
    if (simulate_peak(N, N, prof) <= lim) return N;
    int lo = 1, hi = N;   // peak(lo) fits (M = 1 stores nothing), peak(hi) does not
    while (hi - lo > 1) {
        const int mid = lo + (hi - lo) / 2;
        if (simulate_peak(N, mid, prof) <= lim) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The uniform planning ratio with which plan_slots gives exactly M slots (0 if M = 1).
double ratio_for_slots(int N, size_t mem_budget, size_t S, int M)
{
    if (M <= 1) return 0.0;
    double slot = std::floor((double)mem_budget / (double)(M - 1)) - 512.0;
    if (slot < 1.0) slot = 1.0;
    double F = (double)S / slot;
    for (int it = 0; it < 64 && plan_slots(N, mem_budget, S, true, F) < M; ++it) F *= 1.0 + 1e-9;
    for (int it = 0; it < 64 && plan_slots(N, mem_budget, S, true, F) > M; ++it) F *= 1.0 - 1e-9;
    return F;
}

int validate_model(const wv_model *m, Setup &su)
{
    if (!m || (m->ndim != 2 && m->ndim != 3)) return WV_EINVAL;
    if (m->space_order < 2 || m->space_order > 16 || (m->space_order & 1)) return WV_EINVAL;
    if (m->nbl < 0 || m->nt < 1 || !(m->dt > 0) || !(m->vmax > 0) || !std::isfinite(m->vmax) || !m->vel)
        return WV_EINVAL;
    if (m->time_order != 0 && m->time_order != 2 && m->time_order != 4) return WV_EINVAL;
    long long P = 1;
    for (int a = 0; a < m->ndim; ++a) {
        if (m->n[a] < 1 || !(m->h[a] > 0) || !std::isfinite(m->h[a])) return WV_EINVAL;
        su.N[a] = m->n[a] + 2 * m->nbl;
        P *= su.N[a];
    }
    if (P >= (1LL << 31)) return WV_EINVAL;
    su.P = P;
    su.ndim = m->ndim;
    const double lim = cfl_limit(m->ndim, m->h, m->space_order, m->vmax, m->time_order == 4 ? 4 : 2);
    if (!(lim > 0)) return WV_EINVAL;
    if (m->dt > lim * (1.0 + 1e-12)) return WV_ECFL;
    Grid &g = su.g;
    std::memset(&g, 0, sizeof(g));
    g.ndim = m->ndim;
    g.K = m->space_order / 2;
    g.time_order = m->time_order == 4 ? 4 : 2;
    double a[kMaxK + 1];
    fd_weights(g.K, a);
    // array axes: x = model axis 0; 3-D: y = axis 1, z = axis 2; 2-D: z = axis 1
    const int ax_y = m->ndim == 3 ? 1 : -1, ax_z = m->ndim == 3 ? 2 : 1;
    g.nx = su.N[0];
    g.ny = ax_y >= 0 ? su.N[ax_y] : 1;
    g.nz = su.N[ax_z];
    g.px = m->ndim == 3 ? (g.nx + 31) / 32 * 32 : g.nx;
    su.Pf = (long long)g.px * g.ny * g.nz;
    if (su.Pf >= (1LL << 31)) return WV_EINVAL;
    g.P = su.Pf;
    const int axes[3] = {0, ax_y, ax_z};
    float *cc[3] = {g.cx, g.cy, g.cz};
    float *dd[3] = {&g.dampx, &g.dampy, &g.dampz};
    for (int t = 0; t < 3; ++t) {
        const int ax = axes[t];
        if (ax < 0) {
            g.ix0[t] = 0;
            g.ix1[t] = 0;
            g.cf2[t] = 0.0f;
            *dd[t] = 0.0f;
            continue;
        }
        const double h = m->h[ax];
        for (int k = 1; k <= g.K; ++k) cc[t][k] = (float)(a[k] / (h * h));
        double far = 0.0;
        for (int k = 2; k <= g.K; ++k) far += (double)cc[t][k];
        g.cf2[t] = (float)(2.0 * far);
        if (t > 0) cc[t][0] = (float)((m->h[0] * m->h[0]) / (h * h));
        g.ix0[t] = m->nbl;
        g.ix1[t] = m->nbl + m->n[ax] - 1;
        if (m->nbl > 0) {
            const double smax = 3.0 * m->vmax * std::log(1000.0) / (2.0 * m->nbl * h);
            *dd[t] = (float)(0.5 * m->dt * smax / ((double)m->nbl * m->nbl));
        } else {
            *dd[t] = 0.0f;
        }
    }
    return WV_OK;
}

// Multilinear weights of one position (metres from the first interior point).
int point_weights(const wv_model *m, const Setup &su, const double *xyz, int *idx, float *wt)
{
    int i0[3] = {0, 0, 0};
    double fr[3] = {0, 0, 0};
    for (int d = 0; d < m->ndim; ++d) {
        const double gpos = xyz[d] / m->h[d] + (double)m->nbl;
        if (!(gpos >= 0.0) || gpos > (double)(su.N[d] - 1)) return WV_EINVAL;
        int i = (int)std::floor(gpos);
        if (i > su.N[d] - 2) i = su.N[d] - 2;
        if (i < 0) i = 0;
        i0[d] = i;
        fr[d] = gpos - i;
    }
    const int nc = m->ndim == 3 ? 8 : 4;
    for (int c = 0; c < nc; ++c) {
        long long p = 0, stride = 1;
        double w = 1.0;
        for (int d = 0; d < m->ndim; ++d) {
            const int bit = (c >> d) & 1;
            const int ii = std::min(i0[d] + bit, su.N[d] - 1);
            p += (long long)ii * stride;
            stride *= d == 0 ? su.g.px : su.N[d];   // pitched field arrays
            w *= bit ? fr[d] : 1.0 - fr[d];
        }
        idx[c] = (int)p;
        wt[c] = (float)w;
    }
    return WV_OK;
}

// gather tables plus the transposed (scatter) table with unique points
int build_sparse(const wv_model *m, const Setup &su, int npt, const double *xyz, bool shared_col,
                 std::vector<int> &gidx, std::vector<float> &gwt, std::vector<int> &pts, std::vector<int> &start,
                 std::vector<int> &col, std::vector<float> &swt, int &nc_out)
{
    const int nc_all = m->ndim == 3 ? 8 : 4;
    std::vector<int> gi((size_t)npt * nc_all, 0);
    std::vector<float> gw((size_t)npt * nc_all, 0.0f);
    for (int r = 0; r < npt; ++r) {
        const int rc = point_weights(m, su, xyz + (size_t)r * m->ndim, &gi[(size_t)r * nc_all], &gw[(size_t)r * nc_all]);
        if (rc) return rc;
    }
    // A corner of weight zero (a point on a grid line or node) adds nothing to a gather
    // or a scatter: the tables keep the others, in corner order, each point padded to the
    // largest count with zero weights at its first corner (so a sum takes the same
    // values in the same order, without the zero terms).
    int nc = 1;
    for (int r = 0; r < npt; ++r) {
        int k = 0;
        for (int c = 0; c < nc_all; ++c) k += gw[(size_t)r * nc_all + c] != 0.0f;
        nc = std::max(nc, k);
    }
    gidx.assign((size_t)npt * nc, 0);
    gwt.assign((size_t)npt * nc, 0.0f);
    for (int r = 0; r < npt; ++r) {
        int j = 0;
        for (int c = 0; c < nc_all; ++c) {
            const size_t a = (size_t)r * nc_all + c;
            if (gw[a] == 0.0f) continue;
            gidx[(size_t)r * nc + j] = gi[a];
            gwt[(size_t)r * nc + j] = gw[a];
            ++j;
        }
        for (; j < nc; ++j) gidx[(size_t)r * nc + j] = gi[(size_t)r * nc_all];
    }
    nc_out = nc;
    // entries sorted by (point, column, corner) for a fixed summation order
    struct E { int p, col, c; float w; };
    std::vector<E> es;
    es.reserve((size_t)npt * nc);
    for (int r = 0; r < npt; ++r)
        for (int c = 0; c < nc; ++c)
            if (gwt[(size_t)r * nc + c] != 0.0f)
                es.push_back({gidx[(size_t)r * nc + c], shared_col ? 0 : r, c, gwt[(size_t)r * nc + c]});
    std::sort(es.begin(), es.end(), [](const E &a, const E &b) {
        if (a.p != b.p) return a.p < b.p;
        if (a.col != b.col) return a.col < b.col;
        return a.c < b.c;
    });
    pts.clear();
    start.clear();
    col.clear();
    swt.clear();
    for (size_t i = 0; i < es.size(); ++i) {
        if (i == 0 || es[i].p != es[i - 1].p) {
            pts.push_back(es[i].p);
            start.push_back((int)col.size());
        }
        col.push_back(es[i].col);
        swt.push_back(es[i].w);
    }
    start.push_back((int)col.size());
    return WV_OK;
}

int prepare(const wv_model *m, const wv_geom *geo, Setup &su)
{
    // the launch wrappers report hipGetLastError(); drop any error a previous,
    // unrelated runtime call of this thread left behind
    (void)hipGetLastError();
    int rc = validate_model(m, su);
    if (rc) return rc;
    if (!geo || geo->nsrc < 1 || geo->nrec < 1 || !geo->src_xyz || !geo->rec_xyz || !geo->wavelet)
        return WV_EINVAL;
    rc = build_sparse(m, su, geo->nsrc, geo->src_xyz, true, su.src_gidx, su.src_gwt, su.src_pts, su.src_start,
                      su.src_col, su.src_swt, su.src_nc);
    if (rc) return rc;
    return build_sparse(m, su, geo->nrec, geo->rec_xyz, false, su.rec_gidx, su.rec_gwt, su.rec_pts, su.rec_start,
                        su.rec_col, su.rec_swt, su.rec_nc);
}

size_t tab_bytes(const Setup &su, bool rec)
{
    const size_t ng = rec ? su.rec_gidx.size() : su.src_gidx.size();
    const size_t np = rec ? su.rec_pts.size() : su.src_pts.size();
    const size_t ne = rec ? su.rec_col.size() : su.src_col.size();
    return align_up(ng * 4, 256) * 2 + align_up(np * 4, 256) + align_up((np + 1) * 4, 256) +
           align_up(ne * 4, 256) * 2;
}

// Largest stream one wavefield can take (the arena of a compressibility run).
size_t field_stream_max(const Setup &su)
{
    const int cdims[3] = {su.g.nx, su.ndim == 3 ? su.g.ny : su.g.nz, su.ndim == 3 ? su.g.nz : 1};
    return codec_max_bytes(codec_dims(su.ndim, cdims, su.g.px)) + 256;
}

Layout plan_layout(const wv_model *m, const wv_geom *geo, const Setup &su, int op, size_t budget)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const size_t fb = (size_t)su.Pf * 4;
    L.bk = take(kBk);
    L.U0 = take(fb);
    L.U1 = take(fb);
    L.W = take(fb);
    L.Z = take(fb);
    const bool ot4 = su.g.time_order == 4;
    if (ot4) L.V = take(fb);                    // OT4: v = w lap u (first pass of a step)
    L.src_tab = take(tab_bytes(su, false));
    L.rec_tab = take(tab_bytes(su, true));
    const size_t data_bytes = (size_t)(m->nt + 1) * geo->nrec * 4;
    if (op == WV_OP_GRADIENT) {
        L.L0 = take(fb);
        L.L1 = take(fb);
        L.UB = take(fb);
        L.DB = take(fb);
        if (ot4) L.VU = take(fb);               // OT4 adjoint: w lap u^k for the gradient term
        // 3-D OT2 adjoint: the gradient term an even step carries to the next one
        if (!ot4 && su.ndim == 3) L.CR = take(fb);
        L.res = take(data_bytes);
        L.dsim = take(data_bytes);
        L.partials = take(kParts * 8);
        const int cdims[3] = {su.g.nx, su.ndim == 3 ? su.g.ny : su.g.nz, su.ndim == 3 ? su.g.nz : 1};
        const CodecDims cd = codec_dims(su.ndim, cdims, su.g.px);
        L.nchunks_max = cd.nchunks;
        L.enc = take(encode_work_bytes(cd, true));   // the encoder's chunk counts, offsets, slots
        L.offs_n = 2 * (m->nt + 3);
        L.offs = take((size_t)L.offs_n * 8);
        L.sizes = take((size_t)(m->nt + 1) * 8);   // stream bytes of u^k for each stored state k
        L.arena_bytes = align_up(budget, 256);
        L.arena = take(L.arena_bytes);
    }
    L.total = off;
    return L;
}

struct Dev {
    uint8_t *base;
    Layout L;
    Sparse src, rec;
    float *U[2], *Lm[2], *W, *Z, *UB, *DB, *V = nullptr, *VU = nullptr, *CR = nullptr;
    unsigned *err;
    double *misfit;
    unsigned long long *stats;
    uint64_t *zero, *probe_next, *offs, *sizes;
    uint8_t *enc;
    uint8_t *arena;
    float *res, *dsim;
    double *partials;
};

template <typename T>
T *at(uint8_t *b, size_t o) { return reinterpret_cast<T *>(b + o); }

int upload_tables(Dev &d, const Setup &su, hipStream_t s)
{
    // pack both tables into one host buffer, one copy
    std::vector<uint8_t> host(d.L.src_tab < d.L.rec_tab ? (d.L.rec_tab - d.L.src_tab) + tab_bytes(su, true) : 0);
    auto place = [&](size_t tab_off, bool rec, Sparse &sp) {
        const std::vector<int> &gidx = rec ? su.rec_gidx : su.src_gidx;
        const std::vector<float> &gwt = rec ? su.rec_gwt : su.src_gwt;
        const std::vector<int> &pts = rec ? su.rec_pts : su.src_pts;
        const std::vector<int> &start = rec ? su.rec_start : su.src_start;
        const std::vector<int> &col = rec ? su.rec_col : su.src_col;
        const std::vector<float> &swt = rec ? su.rec_swt : su.src_swt;
        size_t o = tab_off - d.L.src_tab;
        auto put = [&](const void *src, size_t bytes) {
            std::memcpy(host.data() + o, src, bytes);
            const size_t here = o;
            o = align_up(o + bytes, 256);
            return d.base + d.L.src_tab + here;
        };
        const int nc = rec ? su.rec_nc : su.src_nc;
        sp.n = (int)(gidx.size() / nc);
        sp.nc = nc;
        sp.g_idx = (const int *)put(gidx.data(), gidx.size() * 4);
        sp.g_wt = (const float *)put(gwt.data(), gwt.size() * 4);
        sp.npts = (int)pts.size();
        sp.s_pts = (const int *)put(pts.data(), pts.size() * 4);
        sp.s_start = (const int *)put(start.data(), start.size() * 4);
        sp.s_col = (const int *)put(col.data(), col.size() * 4);
        sp.s_wt = (const float *)put(swt.data(), swt.size() * 4);
    };
    place(d.L.src_tab, false, d.src);
    place(d.L.rec_tab, true, d.rec);
    HIPCHK(hipMemcpyAsync(d.base + d.L.src_tab, host.data(), host.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return WV_OK;
}

int bind(Dev &d, void *ws, size_t ws_bytes, const Layout &L, int op)
{
    if (!ws || ws_bytes < L.total) return WV_ENOMEM;
    if (((uintptr_t)ws) & 255) return WV_EINVAL;
    d.base = (uint8_t *)ws;
    d.L = L;
    d.U[0] = at<float>(d.base, L.U0);
    d.U[1] = at<float>(d.base, L.U1);
    if (L.V) d.V = at<float>(d.base, L.V);
    d.W = at<float>(d.base, L.W);
    d.Z = at<float>(d.base, L.Z);
    d.err = at<unsigned>(d.base, L.bk + kErr);
    d.misfit = at<double>(d.base, L.bk + kMisfit);
    d.stats = at<unsigned long long>(d.base, L.bk + kStats);
    d.zero = at<uint64_t>(d.base, L.bk + kZero);
    d.probe_next = at<uint64_t>(d.base, L.bk + kProbeNext);
    if (op == WV_OP_GRADIENT) {
        d.Lm[0] = at<float>(d.base, L.L0);
        d.Lm[1] = at<float>(d.base, L.L1);
        if (L.VU) d.VU = at<float>(d.base, L.VU);
        if (L.CR) d.CR = at<float>(d.base, L.CR);
        d.UB = at<float>(d.base, L.UB);
        d.DB = at<float>(d.base, L.DB);
        d.res = at<float>(d.base, L.res);
        d.dsim = at<float>(d.base, L.dsim);
        d.partials = at<double>(d.base, L.partials);
        d.enc = at<uint8_t>(d.base, L.enc);
        d.offs = at<uint64_t>(d.base, L.offs);
        d.sizes = at<uint64_t>(d.base, L.sizes);
        d.arena = at<uint8_t>(d.base, L.arena);
    }
    return WV_OK;
}

int read_err(Dev &d, hipStream_t s, unsigned *out)
{
    HIPCHK(hipMemcpyAsync(out, d.err, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return WV_OK;
}

// Common set-up: zero the bookkeeping block, compute w, validate the velocity.
int start(Dev &d, const wv_model *m, const Setup &su, hipStream_t s)
{
    HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk), kBk / 8, 0, s));
    int rc = upload_tables(d, su, s);
    if (rc) return rc;
    HIPCHK(launch_setup_w(su.g, m->vel, d.W, m->dt, m->vmax, d.err, s));
    // every field array starts at zero: kernels write only the nx valid columns of a
    // pitched row, so the pad columns keep this zero for the whole call (and whole-array
    // scans such as the finiteness check read no stale workspace bytes)
    float *const fields[] = {d.Z, d.U[0], d.U[1], d.Lm[0], d.Lm[1], d.UB, d.DB, d.V, d.VU};
    for (float *f : fields)
        if (f) HIPCHK(launch_fill_f32(f, su.Pf, 0.0f, s));
    unsigned e = 0;
    rc = read_err(d, s, &e);
    if (rc) return rc;
    return e ? WV_EINVAL : WV_OK;
}

// The forward state x_k = (u^k, d^k).  It lives either in the working buffers
// (U[cur], D) or, right after a restore, in place at its source: the zero field for
// x_0, the checkpoint slot itself (uncompressed) or the decoded base pair
// (compressed).  The next step reads it there and writes the working buffers, so a
// restore moves no data.
// Device timing with one event pair per timed region (a schedule action, or one stencil
// launch), read after the final sync.
struct ActionTimer {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
    ~ActionTimer()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    int begin(int k)
    {
        if (!on) return WV_OK;
        if (used + 2 > ev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                ev.push_back(e);
            }
        }
        kind.push_back(k);
        HIPCHK(hipEventRecord(ev[used], s));
        return WV_OK;
    }
    int end()
    {
        if (!on) return WV_OK;
        HIPCHK(hipEventRecord(ev[used + 1], s));
        used += 2;
        return WV_OK;
    }
    // a fresh event pair of kind k for a launch that records it itself ({} when off)
    int pair(int k, LaunchEvents *le)
    {
        *le = LaunchEvents{};
        if (!on) return WV_OK;
        if (used + 2 > ev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                ev.push_back(e);
            }
        }
        kind.push_back(k);
        le->start = ev[used];
        le->stop = ev[used + 1];
        used += 2;
        return WV_OK;
    }
    // after a sync: accumulate per-kind milliseconds (kinds 1..5 = action codes)
    int totals(double *ms)
    {
        for (size_t i = 0; i < used / 2; ++i) {
            float t = 0.0f;
            HIPCHK(hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]));
            ms[kind[i]] += t;
        }
        return WV_OK;
    }
};

// Forward state x_n = (u^n, u^{n-1}).  The two levels may live anywhere (a
// checkpoint slot, the zero field, the decoded pair): a step writes the work buffer
// that does not hold u^n, which is in place over u^{n-1} once both levels are in the
// work buffers, so restored states are only ever read.
struct Fwd {
    Dev &d;
    const Setup &su;
    const wv_geom *geo;
    hipStream_t s;
    const float *u = nullptr, *up = nullptr;   // u^n, u^{n-1}
    ActionTimer *kt = nullptr;                  // optional per-launch timing of the stencil (kind 0)
    // 2-D: the data row of u^n not gathered yet; the next step's launch gathers it, or
    // flush() after the last step of a run of steps
    float *pend = nullptr;
    void at(const float *cur, const float *prev)
    {
        u = cur;
        up = prev;
    }
    // dest (nullable): where u^{n+1} goes instead of a work level (a checkpoint slot)
    int step(int n, float *data_row, float *dest = nullptr)
    {
        float *out = dest ? dest : ((u == d.U[0]) ? d.U[1] : d.U[0]);
        int rc;
        LaunchEvents le;
        if (kt && (rc = kt->pair(0, &le))) return rc;
        if (su.g.time_order == 4) {
            HIPCHK(launch_lapw(su.g, u, d.V, d.W, s, le));
            if (kt && (rc = kt->pair(0, &le))) return rc;
            HIPCHK(launch_ot4_update(su.g, d.V, u, up, out, d.W, nullptr, nullptr, nullptr, 0.0, s, le));
            HIPCHK(launch_inject_src(su.g, d.src, geo->wavelet, n, d.W, out, s));
        } else if (su.ndim == 2) {
            // the step's own launch injects the source sample and gathers the previous
            // step's receivers
            HIPCHK(launch_fwd_step(su.g, u, up, out, d.W, s, le, &d.src, geo->wavelet + n, pend ? &d.rec : nullptr,
                                   pend));
            pend = nullptr;
        } else {
            HIPCHK(launch_fwd_step(su.g, u, up, out, d.W, s, le));
            HIPCHK(launch_inject_src(su.g, d.src, geo->wavelet, n, d.W, out, s));
        }
        up = u;
        u = out;
        if (data_row) {
            if (su.ndim == 2 && su.g.time_order != 4) pend = data_row;
            else HIPCHK(launch_gather(d.rec, u, data_row, s));
        }
        return WV_OK;
    }
    // gathers the pending data row of the current level
    int flush()
    {
        if (pend) HIPCHK(launch_gather(d.rec, u, pend, s));
        pend = nullptr;
        return WV_OK;
    }
};

double gradient_scale(const wv_model *m) { return -1.0 / (m->dt * m->dt); }

}  // namespace

// =================================================================== C ABI

extern "C" {

const char *wv_strerror(int code)
{
    switch (code) {
    case WV_OK: return "ok";
    case WV_EINVAL: return "invalid argument";
    case WV_ECFL: return "time step above the stability limit";
    case WV_EBUDGET: return "memory budget too small";
    case WV_EARENA: return "compressed checkpoints overflowed the memory budget";
    case WV_ENOMEM: return "workspace too small";
    case WV_EHIP: return "HIP runtime error";
    case WV_EUNSTABLE: return "non-finite wavefield";
    case WV_ENOTIMPL: return "not implemented";
    case WV_ECAP: return "output buffer too small";
    case WV_ETIMEOUT: return "request not finished";
    default: return "unknown error";
    }
}

const char *wv_version(void) { return "wv 0.1 gfx950"; }

const char *wv_last_error(void) { return g_detail; }

double wv_cfl_dt(int ndim, const double *h, int space_order, double vmax)
{
    if (!h) return -1.0;
    return cfl_limit(ndim, h, space_order, vmax);
}

long long wv_field_elements(const wv_model *m)
{
    Setup su;
    if (validate_model(m, su)) return 0;
    return su.Pf;
}

double wv_cfl_dt_to(int ndim, const double *h, int space_order, double vmax, int time_order)
{
    if (!h || (time_order != 2 && time_order != 4)) return -1.0;
    return cfl_limit(ndim, h, space_order, vmax, time_order);
}

long wv_schedule_forward_steps(int nt, int M)
{
    if (nt < 0 || M < 1) return -1;
    return (long)forward_steps(nt, M);
}

int wv_plan(int nt, long long points, size_t mem_budget, const double *profile, int nprofile, int *slots,
            double *ratio_hint)
{
    if (nt < 1 || points < 1 || !profile || nprofile != kProfile || !slots || !ratio_hint) return WV_EINVAL;
    if (!profile_valid(profile)) return WV_EINVAL;
    const int M = plan_slots_profile(nt, mem_budget, profile);
    *slots = M;
    *ratio_hint = ratio_for_slots(nt, mem_budget, (size_t)points * 8, M);
    return WV_OK;
}

int wv_predict(int nt, long long points, size_t mem_budget, int compressed, const wv_costs *costs,
               wv_prediction *out)
{
    if (nt < 1 || points < 1 || !costs || !out) return WV_EINVAL;
    if (compressed && !(costs->ratio > 0)) return WV_EINVAL;
    const size_t S = compressed || !(costs->slot_bytes > 0) ? (size_t)points * 8 : (size_t)costs->slot_bytes;
    const int M = plan_slots(nt, mem_budget, S, compressed != 0, compressed ? costs->ratio : 1.0);
    if (M < 1) return WV_EBUDGET;
    std::vector<int32_t> acts;
    make_schedule(nt, M, compressed == 0, acts);
    const DryRun r = dry_run(acts, M, compressed != 0);
    std::memset(out, 0, sizeof(*out));
    out->slots = M;
    out->advances = r.advances;
    out->stores = r.stores;
    out->fields = r.fields;
    out->decodes = r.decodes;
    out->ms_forward = costs->c_f * (double)r.advances;
    out->ms_adjoint = costs->c_r * (double)r.reverses;
    out->ms_store = (compressed ? costs->t_c : costs->t_copy) * (double)r.fields;
    out->ms_restore = compressed ? costs->t_d * (double)r.decodes : 0.0;
    out->ms_total = out->ms_forward + out->ms_adjoint + out->ms_store + out->ms_restore;
    out->ms_full_storage = (costs->c_f + costs->c_r) * (double)nt;
    return WV_OK;
}

int wv_choose(int nt, long long points, size_t mem_budget, const wv_costs *plain, const wv_costs *compressed,
              const double *profile, int nprofile, wv_choice *out)
{
    if (nt < 1 || points < 1 || !plain || !compressed || !out) return WV_EINVAL;
    if (profile && nprofile != kProfile) return WV_EINVAL;
    const bool use_profile = profile && profile_valid(profile);
    if (!use_profile && !(compressed->ratio > 0)) return WV_EINVAL;
    wv_prediction pp{}, pc{};
    int rc = wv_predict(nt, points, mem_budget, 0, plain, &pp);
    if (rc) return rc;
    wv_costs cc = *compressed;
    if (use_profile) {
        const int M = plan_slots_profile(nt, mem_budget, profile);
        cc.ratio = M > 1 ? ratio_for_slots(nt, mem_budget, (size_t)points * 8, M) : 1.0;
    }
    if ((rc = wv_predict(nt, points, mem_budget, 1, &cc, &pc))) return rc;
    std::memset(out, 0, sizeof(*out));
    out->ms_plain = pp.ms_total;
    out->ms_compressed = pc.ms_total;
    out->compressed = pc.ms_total < pp.ms_total ? 1 : 0;
    out->slots = out->compressed ? pc.slots : pp.slots;
    out->ratio_hint = out->compressed ? cc.ratio : 0.0;
    return WV_OK;
}

int wv_schedule(int nt, int M, int write_min, int32_t *actions, size_t cap, size_t *n_actions)
{
    if (nt < 0 || M < 1 || !n_actions) return WV_EINVAL;
    std::vector<int32_t> a;
    make_schedule(nt, M, write_min != 0, a);
    *n_actions = a.size() / 3;
    if (a.size() / 3 > cap) return WV_ECAP;
    if (!a.empty()) std::memcpy(actions, a.data(), a.size() * 4);
    return WV_OK;
}

size_t wv_workspace_bytes(const wv_model *m, const wv_geom *geo, int op, size_t mem_budget)
{
    Setup su;
    if (prepare(m, geo, su)) return 0;
    if (op == WV_OP_COMPRESSIBILITY) return plan_layout(m, geo, su, WV_OP_GRADIENT, field_stream_max(su)).total;
    if (op != WV_OP_FORWARD && op != WV_OP_GRADIENT) return 0;
    return plan_layout(m, geo, su, op, mem_budget).total;
}

int wv_forward(const wv_model *m, const wv_geom *geo, float *data, float *state_out, void *ws, size_t ws_bytes,
               void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Setup su;
    int rc = prepare(m, geo, su);
    if (rc) return rc;
    if (!data) return WV_EINVAL;
    const Layout L = plan_layout(m, geo, su, WV_OP_FORWARD, 0);
    Dev d{};
    if ((rc = bind(d, ws, ws_bytes, L, WV_OP_FORWARD))) return rc;
    if ((rc = start(d, m, su, s))) return rc;
    HIPCHK(launch_fill_f32(data, geo->nrec, 0.0f, s));
    Fwd f{d, su, geo, s};
    f.at(d.Z, d.Z);
    for (int n = 0; n < m->nt; ++n)
        if ((rc = f.step(n, data + (size_t)(n + 1) * geo->nrec))) return rc;
    if ((rc = f.flush())) return rc;
    if (state_out) {
        // pitched solver rows to the caller's dense layout
        const size_t row = (size_t)su.g.nx * 4, pitch = (size_t)su.g.px * 4, rows = (size_t)su.g.ny * su.g.nz;
        HIPCHK(hipMemcpy2DAsync(state_out, row, f.u, pitch, row, rows, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipMemcpy2DAsync(state_out + su.P, row, f.up, pitch, row, rows, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(launch_check_finite(f.u, su.Pf, d.err, s));
    unsigned e = 0;
    if ((rc = read_err(d, s, &e))) return rc;
    return (e & 8u) ? WV_EUNSTABLE : WV_OK;
}

}  // extern "C"

namespace {

struct GradRun {
    const wv_model *m;
    const wv_geom *geo;
    const Setup &su;
    Dev &d;
    hipStream_t s;
    double tol;
    bool misfit_mode;       // compute d_sim and the residual in the first sweep
    bool src_adj_mode;      // adjoint source only (no forward, no gradient)
    const float *dobs = nullptr;
    const float *residual = nullptr;   // given residual (gradient mode)
    float *dsim_out = nullptr;
    float *src_adj = nullptr;
    double *G = nullptr;
    CodecDims cd{};
    size_t S = 0;                      // bytes of one uncompressed checkpoint (two field arrays)
    size_t Sd = 0;                     // 8 bytes per grid point: the dense pair that ratios refer to
    long advances = 0, stores = 0, restores = 0, reverses = 0, decodes = 0, fields = 0;
    // a first attempt that stores every state without a plan: it stops before the reversal
    // if the arena overflowed, and once it is full encodes only the profile's sample states
    bool optimistic = false, arena_full = false;
    long opt_stores = 0;
    // stream bytes of an all-zero field: prefix plus one bit per block
    double empty_field_bytes() const
    {
        return (double)cd.prefix_bytes + 8.0 * (double)((cd.nblocks + 63) / 64);
    }
    int max_depth = 0;

    // encodes f (or f - sub) at the device offset *base; *next receives the end and
    // size_out (nullable) the stream's bytes
    int encode_field(const float *f, const float *sub, uint64_t *base, uint64_t *next, uint64_t *size_out = nullptr)
    {
        HIPCHK(launch_encode(cd, f, sub, tol, d.arena, d.L.arena_bytes, base, next, d.enc, true, d.err, d.stats, s,
                             size_out));
        return WV_OK;
    }
};

int run_gradient(GradRun &R, int M, double ratio_planned, wv_stats *stats, double *misfit_out)
{
    const wv_model *m = R.m;
    Dev &d = R.d;
    hipStream_t s = R.s;
    const int N = m->nt;
    const long long P = R.su.Pf;   // one field array
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));

    float *data = R.misfit_mode ? (R.dsim_out ? R.dsim_out : d.dsim) : nullptr;
    const float *res = R.misfit_mode ? d.res : R.residual;
    Fwd f{d, R.su, R.geo, s};
    f.at(d.Z, d.Z);
    int hot_slot = -1, hot_k = -1;   // checkpoint currently decoded in the base pair
    HIPCHK(launch_fill_f32(d.Lm[0], P, 0.0f, s));
    HIPCHK(launch_fill_f32(d.Lm[1], P, 0.0f, s));
    if (R.G) HIPCHK(launch_fill_f64(R.G, R.su.P, 0.0, s));   // the caller's dense gradient
    HIPCHK(launch_fill_u64(d.offs, d.L.offs_n, 0, s));
    HIPCHK(launch_fill_u64(d.sizes, N + 1, 0, s));
    if (data) HIPCHK(launch_fill_f32(data, R.geo->nrec, 0.0f, s));
    int gathered = 0;
    bool residual_ready = !R.misfit_mode;
    int lc = 0;
    const double gscale = gradient_scale(m);
    std::vector<int32_t> acts;
    if (R.src_adj_mode) {
        for (int k = N; k >= 1; --k) acts.insert(acts.end(), {REVERSE, k, 0});
    } else {
        make_schedule(N, M, !(R.tol > 0), acts);
    }
    int rc = WV_OK;
    const bool comp = R.tol > 0;
    const size_t fb = (size_t)P * 4;
    const size_t nact = acts.size() / 3;
    const std::vector<char> need2 = second_level_needed(acts, M);
    std::vector<char> slot2((size_t)M + 2, 0);   // slot holds both levels
    bool up_pending = false;                    // restored state: u^{k-1} not decoded yet
    bool hot_db = false;                        // DB holds u^{k-1} of the hot checkpoint
    int pend_slot = -1;
    ActionTimer timer, ktimer;
    timer.on = stats && (stats->timing & 1);
    timer.s = s;
    ktimer.on = stats && (stats->timing & 2);
    ktimer.s = s;
    if (ktimer.on) f.kt = &ktimer;
    for (size_t i = 0; i < acts.size() / 3 && rc == WV_OK; ++i) {
        const int op = acts[3 * i], a = acts[3 * i + 1], b = acts[3 * i + 2];
        if (op != FREE && (rc = timer.begin(op))) break;
        switch (op) {
        case ADVANCE:
            if (!f.up) {   // advancing from a restore: the second level is needed now
                if (!up_pending) {
                    rc = WV_EINVAL;   // cannot happen: the scan above marks these checkpoints
                    break;
                }
                if (!hot_db) {
                    // u^{k-1} = u^k - (u^k - u^{k-1})
                    HIPCHK(launch_decode(R.cd, d.arena, d.offs + 2 * pend_slot + 1, d.L.arena_bytes, d.DB, d.UB,
                                         s));
                    hot_db = true;
                    R.decodes++;
                }
                f.up = d.DB;
                up_pending = false;
            }
            {
                // Uncompressed, an advance that ends in the state the next action stores
                // writes that state straight into its slot (and, when the slot keeps both
                // levels and the advance has two steps or more, u^{b-1} too): the store
                // then copies nothing.  Slots are only read afterwards, as after a restore.
                float *dst_last = nullptr, *dst_prev = nullptr;
                if (!comp && i + 1 < nact && acts[3 * (i + 1)] == STORE && acts[3 * (i + 1) + 1] == b &&
                    acts[3 * (i + 1) + 2] >= 1) {
                    float *slot = reinterpret_cast<float *>(d.arena + (size_t)(acts[3 * (i + 1) + 2] - 1) * R.S);
                    // never into the levels the advance starts from (a slot restored and
                    // stored again): those are read while the steps write
                    const bool clash = f.u == slot || f.u == slot + P || f.up == slot || f.up == slot + P;
                    if (!clash) {
                        dst_last = slot;
                        if (need2[i + 1] && b - a >= 2) dst_prev = slot + P;
                    }
                }
                for (int n = a; n < b && rc == WV_OK; ++n) {
                    float *row = (data && n + 1 > gathered) ? data + (size_t)(n + 1) * R.geo->nrec : nullptr;
                    float *dest = n == b - 1 ? dst_last : (n == b - 2 ? dst_prev : nullptr);
                    if ((rc = f.step(n, row, dest))) break;
                    if (row) gathered = n + 1;
                }
                if (rc == WV_OK) rc = f.flush();
            }
            R.advances += b - a;
            break;
        case STORE:
            slot2[b] = need2[i];
            if (need2[i] && !f.up) {
                rc = WV_EINVAL;
                break;
            }
            if (comp) {
                // u^k at offs[2b]; with both levels the increment u^k - u^{k-1} follows at
                // offs[2b+1]; the next slot starts at offs[2b+2]
                const bool skip = R.optimistic && R.arena_full && !profile_sample(N, a);
                if (skip) {
                    // the arena is full: this attempt will stop, and only the profile's
                    // samples are still measured
                } else if (need2[i]) {
                    if ((rc = R.encode_field(f.u, nullptr, d.offs + 2 * b, d.offs + 2 * b + 1, d.sizes + a))) break;
                    if ((rc = R.encode_field(f.u, f.up, d.offs + 2 * b + 1, d.offs + 2 * b + 2))) break;
                } else {
                    if ((rc = R.encode_field(f.u, nullptr, d.offs + 2 * b, d.offs + 2 * b + 2, d.sizes + a))) break;
                }
                if (hot_slot == b) hot_slot = -1;
                if (R.optimistic && !R.arena_full && ++R.opt_stores % 128 == 0) {
                    unsigned e = 0;
                    if ((rc = read_err(d, s, &e))) break;
                    if (e & 4u) R.arena_full = true;
                }
            } else {
                // copy only the levels the advance before did not write in place
                uint8_t *slot = d.arena + (size_t)(b - 1) * R.S;
                if ((const void *)f.u != (const void *)slot)
                    HIPCHK(hipMemcpyAsync(slot, f.u, fb, hipMemcpyDeviceToDevice, s));
                if (need2[i] && (const void *)f.up != (const void *)(slot + fb))
                    HIPCHK(hipMemcpyAsync(slot + fb, f.up, fb, hipMemcpyDeviceToDevice, s));
            }
            R.stores++;
            R.fields += need2[i] ? 2 : 1;
            R.max_depth = std::max(R.max_depth, b);
            break;
        case RESTORE:
            up_pending = false;
            if (b == 0) {
                f.at(d.Z, d.Z);
            } else if (comp) {
                if (hot_slot != b || hot_k != a) {
                    HIPCHK(launch_decode(R.cd, d.arena, d.offs + 2 * b, d.L.arena_bytes, d.UB, nullptr, s));
                    hot_slot = b;
                    hot_k = a;
                    hot_db = false;
                    R.decodes++;
                }
                // u^{k-1} is decoded by the advance that needs it
                f.at(d.UB, nullptr);
                up_pending = slot2[b] != 0;
                pend_slot = b;
            } else {
                const float *slot = (const float *)(d.arena + (size_t)(b - 1) * R.S);
                f.at(slot, slot2[b] ? slot + P : nullptr);
            }
            R.restores++;
            break;
        case FREE:
            break;
        case REVERSE: {
            if (R.optimistic && R.reverses == 0) {
                unsigned e = 0;
                if ((rc = read_err(d, s, &e))) break;
                if (e & 4u) {   // not every state fits: the caller plans from the sizes
                    rc = WV_EARENA;
                    break;
                }
            }
            if (!residual_ready) {
                HIPCHK(launch_check_finite(f.u, P, d.err, s));
                HIPCHK(launch_residual_misfit(data, R.dobs, d.res, (long long)(N + 1) * R.geo->nrec, R.geo->nrec,
                                              d.partials, kParts, d.misfit, s));
                residual_ready = true;
            }
            const float *uk = R.G ? f.u : nullptr;
            LaunchEvents le;
            if ((rc = ktimer.pair(1, &le))) break;
            // lam^{k-1} overwrites lam^{k+1}
            if (R.su.g.time_order == 4) {
                // v_u = w lap u^k; v = w lap lam^k; then the update, which adds both
                // gradient terms, gscale [u^k (v + (w/12) lap v) + v v_u / 12] (the second
                // is the term of the m inside the OT4 operator)
                if (uk) {
                    HIPCHK(launch_lapw(R.su.g, uk, d.VU, d.W, s, le));
                    if ((rc = ktimer.pair(1, &le))) break;
                }
                HIPCHK(launch_lapw(R.su.g, d.Lm[lc], d.V, d.W, s, le));
                if ((rc = ktimer.pair(1, &le))) break;
                HIPCHK(launch_ot4_update(R.su.g, d.V, d.Lm[lc], d.Lm[lc ^ 1], d.Lm[lc ^ 1], d.W, uk, uk ? d.VU : nullptr,
                                         R.G, gscale, s, le));
            } else {
                // 3-D: the steps k = 2j and 2j - 1 update G once between them (the even
                // step carries its term); an odd first step k = N adds its own
                int gm = kGAdd;
                if (uk && d.CR) gm = a % 2 == 0 ? kGCarryOut : (a < N ? kGCarryIn : kGAdd);
                // 2-D: the step's own launch injects the residual row
                const bool fused = R.su.ndim == 2;
                HIPCHK(launch_adj_step(R.su.g, d.Lm[lc], d.Lm[lc ^ 1], d.Lm[lc ^ 1], d.W, uk, R.G, gscale, s, le,
                                       d.CR, gm, fused ? &d.rec : nullptr,
                                       fused ? res + (size_t)a * R.geo->nrec : nullptr));
            }
            if (R.su.g.time_order == 4 || R.su.ndim == 3)
                HIPCHK(launch_inject_res(R.su.g, d.rec, res + (size_t)a * R.geo->nrec, d.W, d.Lm[lc ^ 1], uk, R.G,
                                         gscale, s));
            lc ^= 1;
            if (R.src_adj) HIPCHK(launch_gather_sum(d.src, d.Lm[lc], R.src_adj + (a - 1), s));
            R.reverses++;
            break;
        }
        default:
            rc = WV_EINVAL;
        }
        if (rc == WV_OK && op != FREE) rc = timer.end();
    }
    if (rc) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return rc;
    }
    HIPCHK(hipEventRecord(e1, s));
    unsigned e = 0;
    unsigned long long st[2] = {0, 0};
    double mis = 0.0;
    HIPCHK(hipMemcpyAsync(st, d.stats, sizeof(st), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&mis, d.misfit, sizeof(double), hipMemcpyDeviceToHost, s));
    if ((rc = read_err(d, s, &e))) return rc;
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (misfit_out) *misfit_out = mis;
    double prof[kProfile];
    for (int j = 0; j < kProfile; ++j) prof[j] = 0.0;
    if (comp && stats) {
        // the compressibility profile of this run from the sizes of the states it stored
        std::vector<uint64_t> sz((size_t)N + 1, 0);
        HIPCHK(hipMemcpy(sz.data(), d.sizes, sz.size() * 8, hipMemcpyDeviceToHost));
        profile_from_sizes(sz, N, R.empty_field_bytes(), prof);
    }
    double kind_ms[6] = {0, 0, 0, 0, 0, 0}, kern_ms[6] = {0, 0, 0, 0, 0, 0};
    if (timer.on && (rc = timer.totals(kind_ms))) return rc;
    if (ktimer.on && (rc = ktimer.totals(kern_ms))) return rc;
    if (stats) {
        const int timing = stats->timing;
        std::memset(stats, 0, sizeof(*stats));
        stats->timing = timing;
        stats->ms_forward = kind_ms[ADVANCE];
        stats->ms_adjoint = kind_ms[REVERSE];
        stats->ms_store = kind_ms[STORE];
        stats->ms_restore = kind_ms[RESTORE];
        stats->ms_fwd_kernel = kern_ms[0];
        stats->ms_adj_kernel = kern_ms[1];
        stats->advances = R.advances;
        stats->stores = R.stores;
        stats->fields = R.fields;
        stats->restores = R.restores;
        stats->decodes = R.decodes;
        stats->reverses = R.reverses;
        stats->slots = M;
        const double raw = (double)R.fields * (double)(R.Sd / 2);   // binary32 fields written (dense)
        stats->bytes_stored = comp ? (double)st[0] : raw;
        stats->peak_bytes = comp ? (double)st[1] : (double)R.max_depth * (double)R.S;
        stats->ratio = stats->bytes_stored > 0 ? raw / stats->bytes_stored : 1.0;
        stats->ratio_planned = ratio_planned;
        stats->misfit = mis;
        stats->ms_total = ms;
        for (int j = 0; j < kProfile; ++j) stats->profile[j] = prof[j];
    }
    if (e & 4u) return WV_EARENA;
    if (e & 16u) return WV_EHIP;
    if (e & (2u | 8u)) return WV_EUNSTABLE;
    return WV_OK;
}

// Compression ratio of the final state of a plain forward run (the paper's
// worst-case proxy): encode (u^N, d^N) at the start of the arena.
// A plain forward run of the shot that measures its compressibility: the stream size
// of u^k at the profile's sample steps and the ratio of the final state (u^N and its
// increment), the paper's worst-case proxy.  The arena serves as scratch.
int probe_ratio(GradRun &R, double *ratio, double *prof)
{
    Dev &d = R.d;
    hipStream_t s = R.s;
    const int N = R.m->nt;
    Fwd f{d, R.su, R.geo, s};
    f.at(d.Z, d.Z);
    HIPCHK(launch_fill_u64(d.offs, d.L.offs_n, 0, s));
    HIPCHK(launch_fill_u64(d.sizes, N + 1, 0, s));
    HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk + kStats), 2, 0, s));
    int rc;
    int next_sample = 1;
    for (int n = 0; n < N; ++n) {
        if ((rc = f.step(n, nullptr))) return rc;
        while (next_sample < kProfile && profile_step(N, next_sample) < n + 1) ++next_sample;
        if (next_sample < kProfile && profile_step(N, next_sample) == n + 1) {
            // u^{n+1} at the start of the arena, for its size only
            if ((rc = R.encode_field(f.u, nullptr, d.offs + 2, d.offs + 3, d.sizes + n + 1))) return rc;
            ++next_sample;
        }
    }
    HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk + kStats), 2, 0, s));
    if ((rc = R.encode_field(f.u, nullptr, d.offs + 2, d.offs + 3))) return rc;
    if ((rc = R.encode_field(f.u, f.up, d.offs + 3, d.offs + 4))) return rc;
    unsigned long long st[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(st, d.stats, sizeof(st), hipMemcpyDeviceToHost, s));
    std::vector<uint64_t> sz((size_t)N + 1, 0);
    HIPCHK(hipMemcpyAsync(sz.data(), d.sizes, sz.size() * 8, hipMemcpyDeviceToHost, s));
    unsigned e = 0;
    if ((rc = read_err(d, s, &e))) return rc;
    if (e & 4u) {   // not even one field fits the arena: plan uncompressed-sized slots
        *ratio = 1.0;
        for (int j = 0; j < kProfile; ++j) prof[j] = 0.0;
        HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk), kBk / 8, 0, s));
        return WV_OK;
    }
    if (e) return WV_EUNSTABLE;
    *ratio = st[0] > 0 ? (double)R.Sd / (double)st[0] : 1.0;
    profile_from_sizes(sz, N, R.empty_field_bytes(), prof);
    HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk), kBk / 8, 0, s));
    return WV_OK;
}

constexpr int kArenaRetries = 3;

int gradient_common(const wv_model *m, const wv_geom *geo, const float *residual, const float *dobs,
                    size_t mem_budget, double tol, double ratio_hint, double *misfit, double *grad_m, float *d_sim,
                    wv_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Setup su;
    int rc = prepare(m, geo, su);
    if (rc) return rc;
    if (!grad_m || !(tol >= 0) || !std::isfinite(tol)) return WV_EINVAL;
    const Layout L = plan_layout(m, geo, su, WV_OP_GRADIENT, mem_budget);
    Dev d{};
    if ((rc = bind(d, ws, ws_bytes, L, WV_OP_GRADIENT))) return rc;
    if ((rc = start(d, m, su, s))) return rc;
    GradRun R{m, geo, su, d, s, tol, dobs != nullptr, false};
    R.dobs = dobs;
    R.residual = residual;
    R.dsim_out = d_sim;
    R.G = grad_m;
    const int cdims[3] = {su.g.nx, su.ndim == 3 ? su.g.ny : su.g.nz, su.ndim == 3 ? su.g.nz : 1};
    R.cd = codec_dims(su.ndim, cdims, su.g.px);
    R.S = (size_t)su.Pf * 8;
    R.Sd = (size_t)su.P * 8;
    const int N = m->nt;
    double F = 1.0;
    if (tol > 0) {
        if (ratio_hint > 0) {
            F = ratio_hint;
        } else {
            // First store every state (the compression-only mode): when the arena holds
            // them all this is the run, and no plan is needed.  Otherwise the attempt
            // stops before the reversal, having measured the states' stream sizes (once
            // the arena is full, only the profile's samples), and the call takes the
            // largest slot count whose peak arena use, simulated over the exact schedule
            // with those sizes, fits.
            R.optimistic = true;
            const double Fall = ratio_for_slots(N, mem_budget, R.Sd, N);
            rc = run_gradient(R, N, Fall > 0 ? Fall : 1.0, stats, misfit);
            R.optimistic = false;
            if (rc != WV_EARENA) return rc;
            std::vector<uint64_t> sz((size_t)N + 1, 0);
            HIPCHK(hipMemcpy(sz.data(), d.sizes, sz.size() * 8, hipMemcpyDeviceToHost));
            double prof[kProfile];
            profile_from_sizes(sz, N, R.empty_field_bytes(), prof);
            HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk), kBk / 8, 0, s));
            R.advances = R.stores = R.restores = R.reverses = R.decodes = R.fields = 0;
            R.max_depth = 0;
            if (profile_valid(prof)) {
                const int Mp = plan_slots_profile(N, mem_budget, prof);
                if (Mp > 1) F = ratio_for_slots(N, mem_budget, R.Sd, Mp);
            }
        }
    }
    // A compressed run whose checkpoints outgrow the budget (the planned ratio was too
    // optimistic) is repeated with half the planned ratio, i.e. fewer slots; the last
    // attempt plans with the uncompressed size, which always fits.
    for (int attempt = 0;; ++attempt) {
        // an uncompressed slot is two field arrays; a compressed one is sized from the
        // dense field bytes and the ratio
        const int M = plan_slots(N, mem_budget, tol > 0 ? R.Sd : R.S, tol > 0, F);
        if (M < 1) return WV_EBUDGET;
        rc = run_gradient(R, M, F, stats, misfit);
        if (rc != WV_EARENA || tol <= 0 || F <= 1.0 || attempt >= kArenaRetries) {
            if (stats) stats->retries = attempt;
            return rc;
        }
        F = attempt + 1 == kArenaRetries ? 1.0 : std::max(1.0, F / 2);
        HIPCHK(launch_fill_u64(at<uint64_t>(d.base, d.L.bk), kBk / 8, 0, s));
        R.advances = R.stores = R.restores = R.reverses = R.decodes = R.fields = 0;
        R.max_depth = 0;
    }
}

}  // namespace

extern "C" {

int wv_gradient(const wv_model *m, const wv_geom *geo, const float *residual, size_t mem_budget, double tol,
                double ratio_hint, double *grad_m, wv_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    if (!residual) return WV_EINVAL;
    return gradient_common(m, geo, residual, nullptr, mem_budget, tol, ratio_hint, nullptr, grad_m, nullptr, stats,
                           ws, ws_bytes, stream);
}

int wv_misfit_gradient(const wv_model *m, const wv_geom *geo, const float *d_obs, size_t mem_budget, double tol,
                       double ratio_hint, double *misfit, double *grad_m, float *d_sim, wv_stats *stats, void *ws,
                       size_t ws_bytes, void *stream)
{
    if (!d_obs || !misfit) return WV_EINVAL;
    return gradient_common(m, geo, nullptr, d_obs, mem_budget, tol, ratio_hint, misfit, grad_m, d_sim, stats, ws,
                           ws_bytes, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ batched 2-D shots
namespace {

constexpr size_t kBatchHdr = 16384;   // barrier counters of the persistent launch, bytes

// program steps for the schedule acts, with the solo executor's bookkeeping (which
// buffer holds each level, when the second level is decoded, which data rows the first
// sweep gathers); every shot of the batch runs the same steps
struct BatchPlan {
    std::vector<BatchOp> ops;
    bool valid = true;
    long advances = 0, stores = 0, restores = 0, reverses = 0, decodes = 0, fields = 0;
    int max_depth = 0;
};

BatchPlan build_batch_program(const std::vector<int32_t> &acts, int M, bool comp)
{
    BatchPlan B;
    auto op = [&](int kind, int n, int a, int b, int c, int d, int e) {
        B.ops.push_back(BatchOp{kind, n, a, b, c, d, e});
    };
    const std::vector<char> need2 = second_level_needed(acts, M);
    std::vector<char> slot2((size_t)M + 2, 0);
    int u = kBufZ, up = kBufZ;            // buffers of u^n and u^{n-1} (kBufNone: not decoded yet)
    int hot_slot = -1, hot_k = -1, pend_slot = -1;
    bool up_pending = false, hot_db = false, residual_ready = false;
    int gathered = 0, lc = 0;
    for (size_t i = 0; i < acts.size() / 3; ++i) {
        const int a = acts[3 * i + 1], b = acts[3 * i + 2];
        switch (acts[3 * i]) {
        case ADVANCE:
            if (up == kBufNone) {   // advancing from a restore: decode the second level now
                if (!up_pending) {      // cannot happen: the scan above marks these checkpoints
                    B.ops.clear();
                    B.valid = false;
                    return B;
                }
                if (!hot_db) {
                    op(kOpDec, -1, kBufDB, kBufUB, 0, 2 * pend_slot + 1, 0);
                    hot_db = true;
                    B.decodes++;
                }
                up = kBufDB;
                up_pending = false;
            }
            op(kOpFwd, a, u, up, 0, b, std::max(a, gathered));
            gathered = std::max(gathered, b);
            for (int n = a; n < b; ++n) {   // the buffers the steps leave behind
                const int out = u == kBufU0 ? kBufU1 : kBufU0;
                up = u;
                u = out;
            }
            B.advances += b - a;
            break;
        case STORE:
            slot2[b] = need2[i];
            if (need2[i] && up == kBufNone) {   // cannot happen either
                B.ops.clear();
                B.valid = false;
                return B;
            }
            if (comp) {
                op(kOpEncCount, a, u, need2[i] ? up : kBufNone, 0, 2 * b, 0);
                op(kOpEncEmit, a, u, need2[i] ? up : kBufNone, 0, 2 * b, 0);
                if (hot_slot == b) hot_slot = -1;
            } else {
                op(kOpCopy, -1, u, kBufSlot + 2 * b, 0, 0, 0);
                if (need2[i]) op(kOpCopy, -1, up, kBufSlot + 2 * b + 1, 0, 0, 0);
            }
            B.stores++;
            B.fields += need2[i] ? 2 : 1;
            B.max_depth = std::max(B.max_depth, b);
            break;
        case RESTORE:
            up_pending = false;
            if (b == 0) {
                u = up = kBufZ;
            } else if (comp) {
                if (hot_slot != b || hot_k != a) {
                    op(kOpDec, -1, kBufUB, kBufNone, 0, 2 * b, 0);
                    hot_slot = b;
                    hot_k = a;
                    hot_db = false;
                    B.decodes++;
                }
                u = kBufUB;
                up = kBufNone;
                up_pending = slot2[b] != 0;
                pend_slot = b;
            } else {
                u = kBufSlot + 2 * b;
                up = slot2[b] ? kBufSlot + 2 * b + 1 : kBufNone;
            }
            B.restores++;
            break;
        case REVERSE:
            if (!residual_ready) {
                op(kOpResid, -1, u, 0, 0, 0, 0);
                op(kOpMisfit, -1, 0, 0, 0, 0, 0);
                residual_ready = true;
            }
            // lam^{k-1} overwrites lam^{k+1}
            op(kOpAdj, a, lc ? kBufL1 : kBufL0, lc ? kBufL0 : kBufL1, u, 0, 0);
            lc ^= 1;
            B.reverses++;
            break;
        default:
            break;
        }
    }
    return B;
}

struct BatchShape {
    size_t hdr, desc, ops, shot0, shot_bytes, chunk_off;
    int max_ops;
    size_t total;
};

int batch_setup(int nshots, const wv_model *ms, const wv_geom *gs, size_t budget, std::vector<Setup> &su,
                std::vector<Layout> &L, BatchShape &B)
{
    if (nshots < 1 || nshots > 4096 || !ms || !gs) return WV_EINVAL;
    const wv_model &m0 = ms[0];
    if (m0.ndim != 2 || (m0.time_order != 0 && m0.time_order != 2)) return WV_EINVAL;
    su.assign((size_t)nshots, Setup{});
    L.assign((size_t)nshots, Layout{});
    for (int i = 0; i < nshots; ++i) {
        const wv_model &m = ms[i];
        const bool same = m.ndim == 2 && m.n[0] == m0.n[0] && m.n[1] == m0.n[1] && m.h[0] == m0.h[0] &&
                          m.h[1] == m0.h[1] && m.nbl == m0.nbl && m.space_order == m0.space_order &&
                          m.nt == m0.nt && m.dt == m0.dt && m.vmax == m0.vmax &&
                          (m.time_order == 0 || m.time_order == 2) && gs[i].nrec == gs[0].nrec;
        if (!same) return WV_EINVAL;
        int rc = prepare(&m, &gs[i], su[i]);
        if (rc) return rc;
        L[i] = plan_layout(&m, &gs[i], su[i], WV_OP_GRADIENT, budget);
    }
    const CodecDims cd = codec_dims(2, std::array<int, 3>{su[0].g.nx, su[0].g.nz, 1}.data(), su[0].g.px);
    B.max_ops = 10 * m0.nt + 64;
    B.hdr = 0;
    B.desc = kBatchHdr;
    B.ops = align_up(B.desc + (size_t)nshots * sizeof(BatchShot), 256);
    B.shot0 = align_up(B.ops + (size_t)B.max_ops * sizeof(BatchOp), 256);
    size_t lay = 0;
    for (int i = 0; i < nshots; ++i) lay = std::max(lay, L[i].total);
    B.chunk_off = align_up(lay, 256);
    B.shot_bytes = align_up(B.chunk_off + (size_t)2 * cd.nchunks * 4, 256);
    B.total = B.shot0 + (size_t)nshots * B.shot_bytes;
    return WV_OK;
}

}  // namespace

extern "C" {

size_t wv_batch_workspace_bytes(int nshots, const wv_model *models, const wv_geom *geoms, size_t mem_budget)
{
    std::vector<Setup> su;
    std::vector<Layout> L;
    BatchShape B{};
    if (batch_setup(nshots, models, geoms, mem_budget, su, L, B)) return 0;
    return B.total;
}

int wv_batch_misfit_gradient(int nshots, const wv_model *models, const wv_geom *geoms, const float *const *d_obs,
                             size_t mem_budget, double tol, double ratio_hint, double *misfits,
                             double *const *grad_m, float *const *d_sim, wv_stats *stats, void *ws, size_t ws_bytes,
                             void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    std::vector<Setup> su;
    std::vector<Layout> L;
    BatchShape B{};
    int rc = batch_setup(nshots, models, geoms, mem_budget, su, L, B);
    if (rc) return rc;
    if (!d_obs || !misfits || !grad_m || !(tol >= 0) || !std::isfinite(tol)) return WV_EINVAL;
    for (int i = 0; i < nshots; ++i)
        if (!d_obs[i] || !grad_m[i]) return WV_EINVAL;
    if (!ws || ws_bytes < B.total) return WV_ENOMEM;
    if (((uintptr_t)ws) & 255) return WV_EINVAL;
    uint8_t *base = (uint8_t *)ws;
    const wv_model &m0 = models[0];
    const int N = m0.nt;
    const Grid &g = su[0].g;
    const int cdims[3] = {g.nx, g.nz, 1};
    const CodecDims cd = codec_dims(2, cdims, g.px);
    const int nwg = batch2d_resident_workgroups(g.K);
    if (nwg < 1) return hip_fail(hipErrorInvalidValue, "batch2d_resident_workgroups", __LINE__);
    // per-shot set-up, as a solo call: tables, w, velocity check, zeroed work arrays
    std::vector<Dev> dv((size_t)nshots);
    std::vector<BatchShot> shots((size_t)nshots);
    for (int i = 0; i < nshots; ++i) {
        uint8_t *sb = base + B.shot0 + (size_t)i * B.shot_bytes;
        if ((rc = bind(dv[i], sb, B.shot_bytes, L[i], WV_OP_GRADIENT))) return rc;
        if ((rc = start(dv[i], &models[i], su[i], s))) return rc;
        Dev &d = dv[i];
        BatchShot &S = shots[i];
        S.U[0] = d.U[0];
        S.U[1] = d.U[1];
        S.UB = d.UB;
        S.DB = d.DB;
        S.Lm[0] = d.Lm[0];
        S.Lm[1] = d.Lm[1];
        S.Z = d.Z;
        S.W = d.W;
        S.wavelet = geoms[i].wavelet;
        S.dobs = d_obs[i];
        S.dsim = (d_sim && d_sim[i]) ? d_sim[i] : d.dsim;
        S.res = d.res;
        S.G = grad_m[i];
        S.partials = d.partials;
        S.misfit = d.misfit;
        S.arena = d.arena;
        S.arena_bytes = d.L.arena_bytes;
        S.offs = d.offs;
        S.sizes = d.sizes;
        S.chunk_words = (uint32_t *)(sb + B.chunk_off);
        S.err = d.err;
        S.stats = d.stats;
        S.src = d.src;
        S.rec = d.rec;
    }
    const size_t Sd = (size_t)su[0].P * 8;   // the dense pair that ratios refer to
    const size_t Sp = (size_t)su[0].Pf * 8;  // one uncompressed slot
    double F = 1.0;
    if (tol > 0) {
        if (ratio_hint > 0) {
            F = ratio_hint;
        } else {
            // each shot's compressibility probe; the batch takes the smallest slot count
            int Mmin = N;
            double Fmin = 0.0;
            for (int i = 0; i < nshots; ++i) {
                GradRun R{&models[i], &geoms[i], su[i], dv[i], s, tol, true, false};
                R.cd = cd;
                R.S = Sp;
                R.Sd = Sd;
                double Fi = 1.0, prof[kProfile];
                if ((rc = probe_ratio(R, &Fi, prof))) return rc;
                int Mi = plan_slots(N, mem_budget, Sd, true, Fi);
                if (profile_valid(prof)) Mi = plan_slots_profile(N, mem_budget, prof);
                if (i == 0 || Mi < Mmin) {
                    Mmin = Mi;
                    Fmin = Fi;
                }
            }
            F = Mmin > 1 ? ratio_for_slots(N, mem_budget, Sd, Mmin) : std::max(1.0, Fmin);
        }
    }
    const double gscale = gradient_scale(&m0);
    BatchArgs A{};
    A.g = g;
    A.cd = cd;
    A.shots = reinterpret_cast<const BatchShot *>(base + B.desc);
    A.nshots = nshots;
    A.ops = reinterpret_cast<const BatchOp *>(base + B.ops);
    A.gscale = gscale;
    A.tol = tol;
    {
        int te;
        std::frexp(tol > 0 ? tol : 1.0, &te);
        A.minexp = te - 1;
    }
    A.nrec = geoms[0].nrec;
    A.nt = N;
    // Launch shape.  Every workgroup takes part in every grid barrier, whose cost grows
    // with the number of arrivals, so the grid is no larger than the widest phase needs:
    // a step phase takes one item per z-chunk of a 256-column tile (16 rows, halved down
    // to 4 while the batch has fewer chunks than twice the CU count) plus one gather item
    // per shot, and the codec phases one item per 256-block chunk and field.  Phases
    // with more items loop over them.
    {
        int cus = 0, dev = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        const long long tiles_x = (g.nx + 255) / 256;
        auto chunks = [&](int zl) { return (long long)nshots * tiles_x * ((g.nz + zl - 1) / zl); };
        int zl = 16;
        while (zl > 4 && chunks(zl) < 2LL * cus) zl /= 2;
        A.zlen = zl;
        const long long widest = std::max(chunks(zl) + nshots, (long long)nshots * 2 * cd.nchunks);
        A.nwg = (int)std::min<long long>(nwg, std::max<long long>(widest, 8));
    }
    A.slot_elems = (long long)su[0].Pf * 2;
    A.bar = reinterpret_cast<unsigned *>(base + B.hdr);
    // WV_BATCH_SPIN_LIMIT (for tests of the fallback) lowers the barrier's poll bound
    A.spin_limit = 1u << 18;
    if (const char *sl = std::getenv("WV_BATCH_SPIN_LIMIT")) A.spin_limit = (unsigned)std::strtoul(sl, nullptr, 10);
    for (int i = 0; i < nshots; ++i) {
        A.src_pts = std::max(A.src_pts, shots[i].src.npts);
        A.rec_pts = std::max(A.rec_pts, shots[i].rec.npts);
    }
    HIPCHK(hipMemcpyAsync(base + B.desc, shots.data(), shots.size() * sizeof(BatchShot), hipMemcpyHostToDevice, s));
    int shrinks = 0;   // relaunches with half the workgroups after a barrier gave up
    for (int attempt = 0;; ++attempt) {
        const int M = plan_slots(N, mem_budget, tol > 0 ? Sd : Sp, tol > 0, F);
        if (M < 1) return WV_EBUDGET;
        std::vector<int32_t> acts;
        make_schedule(N, M, !(tol > 0), acts);
        const BatchPlan plan = build_batch_program(acts, M, tol > 0);
        // cannot happen: the program is bounded by the action count, and the executor's
        // bookkeeping always has the levels a step reads
        if (!plan.valid || (int)plan.ops.size() > B.max_ops) return WV_EINVAL;
        A.nops = (int)plan.ops.size();
        for (int i = 0; i < nshots; ++i) {
            Dev &d = dv[i];
            HIPCHK(launch_fill_f32(d.Lm[0], su[i].Pf, 0.0f, s));
            HIPCHK(launch_fill_f32(d.Lm[1], su[i].Pf, 0.0f, s));
            HIPCHK(launch_fill_f64(grad_m[i], su[i].P, 0.0, s));
            HIPCHK(launch_fill_u64(d.offs, d.L.offs_n, 0, s));
            HIPCHK(launch_fill_u64(d.sizes, N + 1, 0, s));
            HIPCHK(launch_fill_f32(shots[i].dsim, geoms[i].nrec, 0.0f, s));
        }
        HIPCHK(launch_fill_u64(reinterpret_cast<uint64_t *>(base + B.hdr), kBatchHdr / 8, 0, s));
        HIPCHK(hipMemcpyAsync(base + B.ops, plan.ops.data(), plan.ops.size() * sizeof(BatchOp),
                              hipMemcpyHostToDevice, s));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, s));
        HIPCHK(launch_batch2d(A, g.K, s));
        HIPCHK(hipEventRecord(e1, s));
        HIPCHK(hipStreamSynchronize(s));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        bool overflow = false, timeout = false, unstable = false;
        for (int i = 0; i < nshots; ++i) {
            Dev &d = dv[i];
            unsigned e = 0;
            unsigned long long st[2] = {0, 0};
            double mis = 0.0;
            HIPCHK(hipMemcpy(&e, d.err, 4, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(st, d.stats, 16, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(&mis, d.misfit, 8, hipMemcpyDeviceToHost));
            misfits[i] = mis;
            overflow |= (e & 4u) != 0;
            timeout |= (e & 16u) != 0;
            unstable |= (e & (2u | 8u)) != 0;
            if (stats) {
                wv_stats &o = stats[i];
                const int timing = o.timing;
                std::memset(&o, 0, sizeof(o));
                o.timing = timing;
                o.advances = plan.advances;
                o.stores = plan.stores;
                o.fields = plan.fields;
                o.restores = plan.restores;
                o.decodes = plan.decodes;
                o.reverses = plan.reverses;
                o.slots = M;
                const double raw = (double)plan.fields * (double)(Sd / 2);
                const bool comp = tol > 0;
                o.bytes_stored = comp ? (double)st[0] : raw;
                o.peak_bytes = comp ? (double)st[1] : (double)plan.max_depth * (double)Sp;
                o.ratio = o.bytes_stored > 0 ? raw / o.bytes_stored : 1.0;
                o.ratio_planned = F;
                o.misfit = mis;
                o.ms_total = ms;
                o.retries = attempt + shrinks;
                if (comp) {
                    std::vector<uint64_t> sz((size_t)N + 1, 0);
                    HIPCHK(hipMemcpy(sz.data(), d.sizes, sz.size() * 8, hipMemcpyDeviceToHost));
                    GradRun R{&models[i], &geoms[i], su[i], dv[i], s, tol, true, false};
                    R.cd = cd;
                    profile_from_sizes(sz, N, R.empty_field_bytes(), o.profile);
                }
            }
        }
        if (timeout && A.nwg >= 128 && shrinks < 2) {
            // a barrier of the persistent launch did not complete (its workgroups could not
            // all be resident beside other streams' work): launch again with half the
            // workgroups, which need half the room (they loop over more work items)
            A.nwg = A.nwg / 16 * 8;
            ++shrinks;
            for (int i = 0; i < nshots; ++i) HIPCHK(launch_fill_u64(at<uint64_t>(dv[i].base, dv[i].L.bk), kBk / 8, 0, s));
            --attempt;
            continue;
        }
        if (timeout) {
            // still not: each shot runs alone instead, in its own region of the workspace,
            // with the same arithmetic and so the same bits
            for (int i = 0; i < nshots; ++i) {
                wv_stats st{};
                if (stats) st.timing = stats[i].timing;
                uint8_t *sb = base + B.shot0 + (size_t)i * B.shot_bytes;
                const int r = wv_misfit_gradient(&models[i], &geoms[i], d_obs[i], mem_budget, tol, ratio_hint,
                                                 &misfits[i], grad_m[i], d_sim ? d_sim[i] : nullptr, &st, sb,
                                                 B.shot_bytes, stream);
                if (r) return r;
                st.retries += 1 + shrinks;   // the aborted batch launches
                if (stats) stats[i] = st;
            }
            return WV_OK;
        }
        if (overflow && tol > 0 && F > 1.0 && attempt < kArenaRetries) {
            F = attempt + 1 == kArenaRetries ? 1.0 : std::max(1.0, F / 2);
            for (int i = 0; i < nshots; ++i) HIPCHK(launch_fill_u64(at<uint64_t>(dv[i].base, dv[i].L.bk), kBk / 8, 0, s));
            continue;
        }
        if (overflow) return WV_EARENA;
        if (unstable) return WV_EUNSTABLE;
        return WV_OK;
    }
}

int wv_misfit_gradient_auto(const wv_model *m, const wv_geom *geo, const float *d_obs, size_t mem_budget, double tol,
                            const wv_costs *plain, const wv_costs *compressed, const double *profile, int nprofile,
                            double *misfit, double *grad_m, float *d_sim, wv_stats *stats, wv_choice *choice,
                            void *ws, size_t ws_bytes, void *stream)
{
    if (!m || !(tol > 0) || !std::isfinite(tol)) return WV_EINVAL;
    const long long points = (long long)(m->n[0] + 2 * m->nbl) * (m->n[1] + 2 * m->nbl) *
                             (m->ndim == 3 ? (long long)(m->n[2] + 2 * m->nbl) : 1LL);
    wv_choice ch{};
    int rc = wv_choose(m->nt, points, mem_budget, plain, compressed, profile, nprofile, &ch);
    if (rc) return rc;
    if (choice) *choice = ch;
    return wv_misfit_gradient(m, geo, d_obs, mem_budget, ch.compressed ? tol : 0.0, ch.compressed ? ch.ratio_hint : 0.0,
                              misfit, grad_m, d_sim, stats, ws, ws_bytes, stream);
}

int wv_adjoint_src(const wv_model *m, const wv_geom *geo, const float *residual, float *src_adj, void *ws,
                   size_t ws_bytes, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Setup su;
    int rc = prepare(m, geo, su);
    if (rc) return rc;
    if (!residual || !src_adj) return WV_EINVAL;
    const Layout L = plan_layout(m, geo, su, WV_OP_GRADIENT, 0);
    Dev d{};
    if ((rc = bind(d, ws, ws_bytes, L, WV_OP_GRADIENT))) return rc;
    if ((rc = start(d, m, su, s))) return rc;
    GradRun R{m, geo, su, d, s, 0.0, false, true};
    R.residual = residual;
    R.src_adj = src_adj;
    R.S = (size_t)su.Pf * 8;
    R.Sd = (size_t)su.P * 8;
    return run_gradient(R, 1, 1.0, nullptr, nullptr);
}

int wv_compressibility(const wv_model *m, const wv_geom *geo, double tol, int stride, size_t *bytes, int cap,
                       int *count, void *ws, size_t ws_bytes, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    Setup su;
    int rc = prepare(m, geo, su);
    if (rc) return rc;
    if (!(tol > 0) || !std::isfinite(tol) || stride < 1 || !bytes || !count || cap < 0) return WV_EINVAL;
    const int nsamp = m->nt / stride;
    if (nsamp > cap) return WV_ECAP;
    const Layout L = plan_layout(m, geo, su, WV_OP_GRADIENT, field_stream_max(su));
    Dev d{};
    if ((rc = bind(d, ws, ws_bytes, L, WV_OP_GRADIENT))) return rc;
    if ((rc = start(d, m, su, s))) return rc;
    GradRun R{m, geo, su, d, s, tol, false, false};
    const int cdims[3] = {su.g.nx, su.ndim == 3 ? su.g.ny : su.g.nz, su.ndim == 3 ? su.g.nz : 1};
    R.cd = codec_dims(su.ndim, cdims, su.g.px);
    R.S = (size_t)su.Pf * 8;
    R.Sd = (size_t)su.P * 8;
    Fwd f{d, su, geo, s};
    f.at(d.Z, d.Z);
    int k = 0;
    for (int n = 0; n < m->nt; ++n) {
        if ((rc = f.step(n, nullptr))) return rc;
        if ((n + 1) % stride == 0) {
            // encode u^{n+1} at the start of the arena; its header holds the stream size
            HIPCHK(launch_fill_u64(d.offs, 2, 0, s));
            if ((rc = R.encode_field(f.u, nullptr, d.offs, d.offs + 1))) return rc;
            uint64_t tot = 0;
            HIPCHK(hipMemcpyAsync(&tot, d.arena + 56, sizeof(tot), hipMemcpyDeviceToHost, s));
            unsigned e = 0;
            if ((rc = read_err(d, s, &e))) return rc;
            if (e & 2u) return WV_EUNSTABLE;
            if (e) return WV_EHIP;
            bytes[k++] = (size_t)tot;
        }
    }
    *count = k;
    return WV_OK;
}

int wv_pad_velocity(int ndim, const int *n, int nbl, const float *vin, float *vout, void *stream)
{
    if ((ndim != 2 && ndim != 3) || !n || nbl < 0 || !vin || !vout) return WV_EINVAL;
    (void)hipGetLastError();
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 1) return WV_EINVAL;
    HIPCHK(launch_pad_velocity(ndim, n, nbl, vin, vout, (hipStream_t)stream));
    return WV_OK;
}

int wv_velocity_gradient(int ndim, const int *n, int nbl, const float *vpad, const double *gm, double *gv,
                         void *stream)
{
    if ((ndim != 2 && ndim != 3) || !n || nbl < 0 || !vpad || !gm || !gv) return WV_EINVAL;
    (void)hipGetLastError();
    for (int a = 0; a < ndim; ++a)
        if (n[a] < 1) return WV_EINVAL;
    HIPCHK(launch_velocity_gradient(ndim, n, nbl, vpad, gm, gv, (hipStream_t)stream));
    return WV_OK;
}

// ------------------------------------------------------------------ codec entry points
namespace {
constexpr size_t kCodecBk = 512;   // err, base word, next word, stats[2]
}

size_t wv_zfpk_workspace_bytes(int ndim, const int *dims)
{
    if ((ndim != 2 && ndim != 3) || !dims) return 0;
    const CodecDims cd = codec_dims(ndim, dims);
    return kCodecBk + encode_work_bytes(cd, true);
}

size_t wv_zfpk_max_bytes(int ndim, const int *dims)
{
    if ((ndim != 2 && ndim != 3) || !dims) return 0;
    return codec_max_bytes(codec_dims(ndim, dims));
}

}  // extern "C"

namespace {

int check_encode_args(const float *field, int ndim, const int *dims, double tol, const void *out,
                      const size_t *nbytes)
{
    if ((ndim != 2 && ndim != 3) || !dims || !field || !out || !nbytes || !(tol > 0) || !std::isfinite(tol))
        return WV_EINVAL;
    for (int a = 0; a < ndim; ++a)
        if (dims[a] < 1) return WV_EINVAL;
    if (((uintptr_t)out) & 7) return WV_EINVAL;
    return WV_OK;
}

// One field through the encoder with its bookkeeping words and work area at b (kCodecBk
// bytes, then encode_work_bytes(cd, staged), 256-byte aligned); the bookkeeping is
// cleared here by a fill kernel and the work area is written before it is read, so b may
// hold anything on entry.  Synchronises the stream.
int encode_one(const float *field, int ndim, const int *dims, double tol, void *out, size_t cap, size_t *nbytes,
               uint8_t *b, bool staged, hipStream_t s)
{
    const CodecDims cd = codec_dims(ndim, dims);
    unsigned *err = (unsigned *)b;
    uint64_t *base = (uint64_t *)(b + 128);
    uint64_t *next = (uint64_t *)(b + 136);
    unsigned long long *st = (unsigned long long *)(b + 192);
    HIPCHK(launch_fill_u64((uint64_t *)b, kCodecBk / 8, 0, s));
    HIPCHK(launch_encode(cd, field, nullptr, tol, (uint8_t *)out, cap, base, next, b + kCodecBk, staged, err, st,
                         s));
    unsigned e = 0;
    unsigned long long tot[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(tot, st, 16, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    *nbytes = (size_t)tot[0];
    if (e & 4u) return WV_ECAP;
    if (e & 2u) return WV_EINVAL;
    return WV_OK;
}

// Scratch of wv_zfpk_encode_noalloc: the encoder's bookkeeping words and its chunk
// counts and offsets (no staging slots: every chunk is encoded twice) in one
// file-scope device array.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code the array's name is only a stand-in, so
// host code never passes it: the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and kept in g_scratch_dev.
constexpr size_t kNoAllocScratchBytes = 192 * 1024;
// chunks whose counts (4 bytes) and offsets (8 bytes) fit, each array padded to 256 bytes
constexpr size_t kNoAllocMaxBlocks = (kNoAllocScratchBytes - kCodecBk - 512) / 12 * kBlocksPerChunk;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

int noalloc_scratch(uint8_t **out)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return WV_EINVAL;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return WV_EHIP;
        g_scratch_dev[dev] = p;
    }
    *out = (uint8_t *)g_scratch_dev[dev];
    return WV_OK;
}

}  // namespace

extern "C" {

int wv_zfpk_encode_noalloc(const float *field, int ndim, const int *dims, double tol, void *out, size_t cap,
                           size_t *nbytes, void *stream)
{
    int rc = check_encode_args(field, ndim, dims, tol, out, nbytes);
    if (rc) return rc;
    (void)hipGetLastError();
    const size_t need = kCodecBk + encode_work_bytes(codec_dims(ndim, dims), false);
    if (need > kNoAllocScratchBytes) {
        std::snprintf(g_detail, sizeof(g_detail),
                      "wv_zfpk_encode_noalloc: %zu bytes of scratch needed, %zu available (at most %zu blocks)",
                      need, kNoAllocScratchBytes, kNoAllocMaxBlocks);
        return WV_ENOMEM;
    }
    uint8_t *b = nullptr;
    if ((rc = noalloc_scratch(&b))) return rc;
    return encode_one(field, ndim, dims, tol, out, cap, nbytes, b, false, (hipStream_t)stream);
}

int wv_zfpk_encode(const float *field, int ndim, const int *dims, double tol, void *out, size_t cap,
                   size_t *nbytes, void *ws, size_t ws_bytes, void *stream)
{
    int rc = check_encode_args(field, ndim, dims, tol, out, nbytes);
    if (rc) return rc;
    (void)hipGetLastError();
    if (!ws || ws_bytes < wv_zfpk_workspace_bytes(ndim, dims) || (((uintptr_t)ws) & 255)) return WV_ENOMEM;
    return encode_one(field, ndim, dims, tol, out, cap, nbytes, (uint8_t *)ws, true, (hipStream_t)stream);
}

int wv_zfpk_decode(const void *in, size_t nbytes, int ndim, const int *dims, float *field, void *stream)
{
    if ((ndim != 2 && ndim != 3) || !dims || !in || !field || (((uintptr_t)in) & 7)) return WV_EINVAL;
    for (int a = 0; a < ndim; ++a)
        if (dims[a] < 1) return WV_EINVAL;
    const CodecDims cd = codec_dims(ndim, dims);
    if (nbytes < (size_t)cd.prefix_bytes) return WV_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();
    // the header must describe exactly this field and fit the readable bytes
    uint8_t h[64];
    HIPCHK(hipMemcpyAsync(h, in, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    uint32_t h32[12];
    uint64_t data_words = 0, total = 0;
    double tol = 0.0;
    std::memcpy(h32, h, sizeof(h32));
    std::memcpy(&tol, h + 24, 8);
    std::memcpy(&data_words, h + 48, 8);
    std::memcpy(&total, h + 56, 8);
    const int want[3] = {cd.dims[0], cd.dims[1], cd.dims[2]};
    bool ok = h32[0] == 0x4B50465Au && h32[1] == 1u && h32[2] == (uint32_t)ndim;
    for (int a = 0; a < 3; ++a) ok = ok && h32[3 + a] == (uint32_t)want[a];
    ok = ok && h32[8] == (uint32_t)cd.nblocks && h32[9] == (uint32_t)cd.nchunks &&
         h32[10] == (uint32_t)kBlocksPerChunk && tol > 0 && std::isfinite(tol);
    ok = ok && data_words <= (uint64_t)(nbytes - (size_t)cd.prefix_bytes) / 8 &&
         total == (uint64_t)cd.prefix_bytes + 8 * data_words && total <= (uint64_t)nbytes;
    if (!ok) return WV_EINVAL;
    HIPCHK(launch_decode(cd, (const uint8_t *)in, nullptr, (uint64_t)total, field, nullptr, s));
    return WV_OK;
}

}  // extern "C"
