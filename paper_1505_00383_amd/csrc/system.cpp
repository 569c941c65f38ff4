// system.cpp -- the system compiler: sparse supports and coefficients to the
// device term tables ("instructions" idx and cff of Table 8 in the paper).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "ph_internal.hpp"

namespace ph {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PH_ENOMEM : PH_EHIP;
}

void free_table(DevTable &t)
{
    if (t.block) (void)hipFree(t.block);
    if (t.u_scratch) (void)hipFree(t.u_scratch);
    t = DevTable{};
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int build_table(const HostSystem &f, const HostSystem *g, DevTable &out)
{
    const int ne = f.n_eq, nv = f.n_var;
    std::vector<int32_t> eq_off(ne + 1, 0), zc_off(ne + 1, 0), zc;
    std::vector<int4> tdesc;
    std::vector<uint32_t> fac;
    std::vector<double> coef;
    int kmax = 0;
    std::vector<char> touched(nv);
    // terms of each equation in order of their number of factors (stable):
    // the tracker evaluates one equation per lane, and equal term shapes at
    // equal positions keep the lanes of a wave on the same path through the
    // sweep; the evaluation kernels are indifferent to the order
    std::vector<int> order;
    auto emit = [&](const HostSystem &s, int i, int sel) {
        order.clear();
        for (int t = s.eq_term_off[i]; t < s.eq_term_off[i + 1]; ++t) order.push_back(t);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return s.term_fac_off[x + 1] - s.term_fac_off[x] < s.term_fac_off[y + 1] - s.term_fac_off[y];
        });
        for (int t : order) {
            int a = s.term_fac_off[t], b = s.term_fac_off[t + 1];
            int4 d;
            d.x = b - a;
            d.y = int(fac.size());
            d.z = sel;
            d.w = 0;
            tdesc.push_back(d);
            kmax = std::max(kmax, b - a);
            for (int q = a; q < b; ++q) {
                uint32_t w = uint32_t(s.fac_var[q]) | (uint32_t(s.fac_exp[q]) << 16);
                if (!touched[s.fac_var[q]]) {
                    w |= FAC_FIRST;
                    touched[s.fac_var[q]] = 1;
                }
                fac.push_back(w);
            }
            for (int c = 0; c < 8; ++c) coef.push_back(s.coef[size_t(t) * 8 + c]);
        }
    };
    for (int i = 0; i < ne; ++i) {
        std::fill(touched.begin(), touched.end(), 0);
        emit(f, i, 0);
        if (g) {
            emit(*g, i, 1);
        } else {
            // g_i = x_i^{d_i} - 1: one term x_i^{d_i} (coefficient 1), one constant
            // -1.  Defined for square systems only; g_i = 0 when d_i = 0.
            int d = f.deg[i];
            if (ne == nv && d > 0) {
                int4 t1;
                t1.x = 1;
                t1.y = int(fac.size());
                t1.z = 1;
                t1.w = 0;
                tdesc.push_back(t1);
                uint32_t w = uint32_t(i) | (uint32_t(d) << 16);
                if (!touched[i]) {
                    w |= FAC_FIRST;
                    touched[i] = 1;
                }
                fac.push_back(w);
                double one[8] = {1, 0, 0, 0, 0, 0, 0, 0};
                coef.insert(coef.end(), one, one + 8);
                kmax = std::max(kmax, 1);
            }
            if (ne == nv && d > 0) {
                int4 t0;
                t0.x = 0;
                t0.y = int(fac.size());
                t0.z = 1;
                t0.w = 0;
                tdesc.push_back(t0);
                double m1[8] = {-1, 0, 0, 0, 0, 0, 0, 0};
                coef.insert(coef.end(), m1, m1 + 8);
            }
        }
        eq_off[i + 1] = int32_t(tdesc.size());
        for (int j = 0; j < nv; ++j)
            if (!touched[j]) zc.push_back(j);
        zc_off[i + 1] = int32_t(zc.size());
    }
    // ---- complex-double fast path: records for terms with k <= 8 and
    // exponents <= 4 (target terms, and explicit start terms); the
    // total-degree start part is evaluated analytically per equation ----
    int emax = 0;
    bool dfast = true;
    auto scan = [&](const HostSystem &sy) {
        for (int t = 0; t < sy.eq_term_off[sy.n_eq]; ++t) {
            int a = sy.term_fac_off[t], b = sy.term_fac_off[t + 1];
            if (b - a > 8) dfast = false;
            for (int q = a; q < b; ++q) emax = std::max(emax, sy.fac_exp[q]);
        }
    };
    scan(f);
    if (g) scan(*g);
    if (emax > 4) dfast = false;
    const int planes = std::max(1, std::min(emax, 4) - 1);  // x, x^2, x^3 as needed
    std::vector<DTerm> dterm;
    std::vector<MTerm> mterm;
    std::vector<int32_t> d_eq_off(ne + 1, 0), d_deg(ne, 0), d_run(1, 0);
    // the double-double staging layout must fit the 160 KB of LDS: planes of
    // 4 nv rows and a ones row, 512 bytes per row
    const bool mfast = dfast && (size_t(planes) * nv * 4 + 4) * 512 <= 160 * 1024;
    if (dfast) {
        // LDS layout per workgroup (doubles, 64 lanes): plane p (x^(p+1)) of
        // variable v, component c at ((p * nv + v) * 2 + c) * 64; then a row
        // of ones (re) and zeros (im).  Double double: rows
        // ((p * nv + v) * 4 + 2 c + limb) * 64, then the ones row {1, 0, 0, 0}.
        const uint32_t ones_off = uint32_t(planes * nv * 2 * 64 * 8);
        const uint32_t ones_off2 = uint32_t(planes * nv * 4 * 64 * 8);
        struct Rec {
            DTerm d;
            MTerm m;
        };
        std::vector<Rec> eqrec;
        auto emit_d = [&](const HostSystem &sy, int i, int sel) {
            for (int t = sy.eq_term_off[i]; t < sy.eq_term_off[i + 1]; ++t) {
                Rec rr;
                DTerm &r = rr.d;
                MTerm &m = rr.m;
                std::memset(&r, 0, sizeof r);
                std::memset(&m, 0, sizeof m);
                r.cre = sy.coef[size_t(t) * 8];
                r.cim = sy.coef[size_t(t) * 8 + 4];
                for (int l = 0; l < 8; ++l) m.c[l] = sy.coef[size_t(t) * 8 + l];
                int a = sy.term_fac_off[t], b = sy.term_fac_off[t + 1];
                r.k = b - a;
                // factors by exponent, largest first: the kernel multiplies
                // x^(a-1) from the power table for a >= 3, x itself for
                // a = 2 and nothing for a = 1, with wave-uniform counts
                int ord[8];
                for (int l = 0; l < r.k; ++l) ord[l] = a + l;
                std::stable_sort(ord, ord + r.k,
                                 [&](int x, int y) { return sy.fac_exp[x] > sy.fac_exp[y]; });
                int m3 = 0, m2 = 0;
                for (int l = 0; l < r.k; ++l) {
                    const int q = ord[l], v = sy.fac_var[q], e = sy.fac_exp[q];
                    const uint32_t poff = e == 1 ? ones_off : uint32_t(((e - 2) * nv + v) * 2 * 64 * 8);
                    r.xo[l] = uint32_t(v) * 2u * 64u * 8u;
                    r.po[l] = poff;
                    r.j2[l] = uint32_t(2 * v);
                    r.a[l] = double(e);
                    m.xo[l] = uint32_t(v) * 4u * 64u * 8u;
                    m.po[l] = e == 1 ? ones_off2 : uint32_t(((e - 2) * nv + v) * 4 * 64 * 8);
                    m.jo[l] = uint32_t(8 * v);
                    m.a[l] = double(e);
                    m3 += e >= 3;
                    m2 += e >= 2;
                }
                r.sel = sel | (m3 << 8) | (m2 << 16);
                m.k = r.k;
                m.sel = r.sel;
                eqrec.push_back(rr);
            }
        };
        d_run.assign(size_t(ne) * DRUN, 0);
        for (int i = 0; i < ne; ++i) {
            eqrec.clear();
            emit_d(f, i, 0);
            if (g) emit_d(*g, i, 1);
            // group the equation's terms by (k, number of factors with
            // a >= 2) so the kernel runs one straight-line loop per group
            // (a stable sort keeps the term order within a group)
            auto grp = [](const DTerm &x) { return drun_group(x.k, (x.sel >> 16) & 15); };
            std::stable_sort(eqrec.begin(), eqrec.end(),
                             [&](const Rec &x, const Rec &y) { return grp(x.d) < grp(y.d); });
            const size_t first = dterm.size();
            for (const Rec &rr : eqrec) {
                dterm.push_back(rr.d);
                mterm.push_back(rr.m);
            }
            for (int gg = 0; gg < DRUN; ++gg) {
                size_t pos = first;
                while (pos < dterm.size() && grp(dterm[pos]) < gg) ++pos;
                d_run[size_t(i) * DRUN + gg] = int32_t(pos);
            }
            d_eq_off[i + 1] = int32_t(dterm.size());
            d_deg[i] = (!g && ne == nv) ? f.deg[i] : 0;
        }
        if (dterm.empty()) {
            dterm.push_back(DTerm{});
            mterm.push_back(MTerm{});
        }
    }
    if (mterm.empty()) mterm.push_back(MTerm{});

    // ---- the unfused design: one slot per term value and per partial,
    // and for every output entry the list of slots summed into it ----
    std::vector<int32_t> u_slot(tdesc.size()), u_off(size_t(ne) * (1 + nv) + 1, 0), u_list;
    {
        std::vector<std::vector<int32_t>> lists(size_t(ne) * (1 + nv));
        int64_t slot = 0;
        for (int i = 0; i < ne; ++i) {
            for (int tt = eq_off[i]; tt < eq_off[i + 1]; ++tt) {
                u_slot[tt] = int32_t(slot);
                lists[i].push_back(int32_t(slot));
                for (int l = 0; l < tdesc[tt].x; ++l) {
                    const int v = fac_var(fac[tdesc[tt].y + l]);
                    lists[size_t(ne) + size_t(i) * nv + v].push_back(int32_t(slot + 1 + l));
                }
                slot += 1 + tdesc[tt].x;
            }
        }
        out.u_slots = slot;
        for (size_t e = 0; e < lists.size(); ++e) {
            u_list.insert(u_list.end(), lists[e].begin(), lists[e].end());
            u_off[e + 1] = int32_t(u_list.size());
        }
        if (u_slot.empty()) u_slot.push_back(0);
        if (u_list.empty()) u_list.push_back(0);
    }

    if (tdesc.empty()) {  // keep every pointer valid
        tdesc.push_back(int4{0, 0, 0, 0});
        coef.resize(8, 0.0);
    }
    if (fac.empty()) fac.push_back(0);
    if (zc.empty()) zc.push_back(0);
    // the tracker's copy of the factor words: eight slots per term (zeros
    // past its factors), so that a term's words are addressed by its index
    // alone and can be read together with its descriptor
    std::vector<uint32_t> fac8(tdesc.size() * 8, 0u);
    for (size_t tt = 0; tt < tdesc.size(); ++tt)
        for (int l = 0; l < tdesc[tt].x && l < 8; ++l) fac8[tt * 8 + l] = fac[tdesc[tt].y + l];

    size_t o_eq = 0;
    size_t o_td = o_eq + align256(eq_off.size() * 4);
    size_t o_fac = o_td + align256(tdesc.size() * sizeof(int4));
    size_t o_cf = o_fac + align256(fac.size() * 4);
    size_t o_zo = o_cf + align256(coef.size() * 8);
    size_t o_zc = o_zo + align256(zc_off.size() * 4);
    size_t o_deo = o_zc + align256(zc.size() * 4);
    size_t o_dt = o_deo + align256(d_eq_off.size() * 4);
    size_t o_mt = o_dt + align256(dterm.size() * sizeof(DTerm));
    size_t o_dd = o_mt + align256(mterm.size() * sizeof(MTerm));
    size_t o_dr = o_dd + align256(d_deg.size() * 4);
    size_t o_us = o_dr + align256(d_run.size() * 4);
    size_t o_uo = o_us + align256(u_slot.size() * 4);
    size_t o_ul = o_uo + align256(u_off.size() * 4);
    size_t o_f8 = o_ul + align256(u_list.size() * 4);
    size_t total = o_f8 + align256(fac8.size() * 4);
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_eq, eq_off.data(), eq_off.size() * 4);
    std::memcpy(host.data() + o_td, tdesc.data(), tdesc.size() * sizeof(int4));
    std::memcpy(host.data() + o_fac, fac.data(), fac.size() * 4);
    std::memcpy(host.data() + o_cf, coef.data(), coef.size() * 8);
    std::memcpy(host.data() + o_zo, zc_off.data(), zc_off.size() * 4);
    std::memcpy(host.data() + o_zc, zc.data(), zc.size() * 4);
    std::memcpy(host.data() + o_deo, d_eq_off.data(), d_eq_off.size() * 4);
    if (!dterm.empty()) std::memcpy(host.data() + o_dt, dterm.data(), dterm.size() * sizeof(DTerm));
    std::memcpy(host.data() + o_mt, mterm.data(), mterm.size() * sizeof(MTerm));
    std::memcpy(host.data() + o_dd, d_deg.data(), d_deg.size() * 4);
    std::memcpy(host.data() + o_dr, d_run.data(), d_run.size() * 4);
    std::memcpy(host.data() + o_us, u_slot.data(), u_slot.size() * 4);
    std::memcpy(host.data() + o_uo, u_off.data(), u_off.size() * 4);
    std::memcpy(host.data() + o_ul, u_list.data(), u_list.size() * 4);
    std::memcpy(host.data() + o_f8, fac8.data(), fac8.size() * 4);
    char *dev = nullptr;
    PH_HIP(hipMalloc(&dev, total));
    hipError_t e = hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "hipMemcpy(term tables)");
    }
    out.n_eq = ne;
    out.n_var = nv;
    out.kmax = kmax;
    out.n_terms = int64_t(tdesc.size());
    out.n_fac = int64_t(fac.size());
    out.block = dev;
    out.eq_off = reinterpret_cast<int32_t *>(dev + o_eq);
    out.tdesc = reinterpret_cast<int4 *>(dev + o_td);
    out.fac = reinterpret_cast<uint32_t *>(dev + o_fac);
    out.fac8 = reinterpret_cast<uint32_t *>(dev + o_f8);
    out.coef = reinterpret_cast<double *>(dev + o_cf);
    out.zc_off = reinterpret_cast<int32_t *>(dev + o_zo);
    out.zc = reinterpret_cast<int32_t *>(dev + o_zc);
    out.emax = emax;
    out.dfast = dfast;
    out.dfast_planes = planes;
    out.d_eq_off = reinterpret_cast<int32_t *>(dev + o_deo);
    out.dterm = reinterpret_cast<DTerm *>(dev + o_dt);
    out.mfast = mfast;
    out.mterm = reinterpret_cast<MTerm *>(dev + o_mt);
    out.d_deg = reinterpret_cast<int32_t *>(dev + o_dd);
    out.d_run = reinterpret_cast<int32_t *>(dev + o_dr);
    out.u_slot = reinterpret_cast<int32_t *>(dev + o_us);
    out.u_off = reinterpret_cast<int32_t *>(dev + o_uo);
    out.u_list = reinterpret_cast<int32_t *>(dev + o_ul);
    return PH_OK;
}

int get_table(const ph_system *target, const ph_system *start, const DevTable **out)
{
    if (!start) {
        *out = &target->total;
        return PH_OK;
    }
    ph_system *t = const_cast<ph_system *>(target);
    std::lock_guard<std::mutex> lk(t->mu);
    auto it = t->with_start.find(start);
    if (it != t->with_start.end()) {
        *out = &it->second;
        return PH_OK;
    }
    DevTable tab;
    int rc = build_table(target->h, &start->h, tab);
    if (rc) return rc;
    auto res = t->with_start.emplace(start, tab);
    *out = &res.first->second;
    return PH_OK;
}

int find_table(const ph_system *target, const ph_system *start, const DevTable **out)
{
    if (!start) {
        *out = &target->total;
        return PH_OK;
    }
    ph_system *t = const_cast<ph_system *>(target);
    std::lock_guard<std::mutex> lk(t->mu);
    auto it = t->with_start.find(start);
    if (it == t->with_start.end())
        return fail(PH_EINVAL, "start system not prepared for this target: call ph_eval_prepare first");
    *out = &it->second;
    return PH_OK;
}

int prepare_unfused(const ph_system *target, DevTable &tab, int prec, int64_t npts)
{
    const int64_t lu = (npts + 63) / 64 * 64;
    const size_t need = (size_t)(tab.n_terms + tab.u_slots) * 2 * prec * lu * sizeof(double);
    std::lock_guard<std::mutex> lk(const_cast<ph_system *>(target)->mu);
    if (tab.u_scratch_bytes >= need) return PH_OK;
    if (tab.u_scratch) {
        // the previous buffer may still be read by work queued on any stream
        PH_HIP(hipDeviceSynchronize());
        (void)hipFree(tab.u_scratch);
        tab.u_scratch = nullptr;
        tab.u_scratch_bytes = 0;
    }
    if (hipMalloc(&tab.u_scratch, need) != hipSuccess) {
        tab.u_scratch = nullptr;
        return fail(PH_ENOMEM, "unfused evaluation: intermediate arrays do not fit");
    }
    tab.u_scratch_bytes = need;
    return PH_OK;
}

void load_eval_cache(ph_system *s)
{
    const char *path = std::getenv("PH_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char tag[16];
        unsigned long long a = 0, b = 0;
        int p = 0, k = 0, w = 0, g = 0;
        double ms = 0;
        // lines "eval <target fp> <start fp> <prec> <kernel> <W> <G> <ms>";
        // other tags (the tracker's) have their own layout
        if (std::sscanf(line, "%15s %llx %llx %d %d %d %d %lf", tag, &a, &b, &p, &k, &w, &g, &ms) == 8 &&
            std::strcmp(tag, "eval") == 0 && a == s->h.fingerprint)
            s->file_cfg[{(uint64_t)b, p}] = EvalCfg{k, w, g};  // the last entry wins
    }
    std::fclose(f);
}

static int validate(int32_t n_eq, int32_t n_var, const int32_t *eq_term_off,
                    const int32_t *term_fac_off, const int32_t *fac_var, const int32_t *fac_exp,
                    const double *coef, int32_t coef_limbs)
{
    if (n_var < 1 || n_eq < 1) return fail(PH_EINVAL, "n_eq and n_var must be >= 1");
    if (n_var > 64 || n_eq > 64) return fail(PH_EUNSUPPORTED, "n_eq and n_var are limited to 64");
    if (n_var > n_eq) return fail(PH_EINVAL, "n_var must not exceed n_eq (least squares needs m >= n)");
    if (!eq_term_off || !term_fac_off || !coef)
        return fail(PH_EINVAL, "null system array");
    if (coef_limbs != 1 && coef_limbs != 2 && coef_limbs != 4)
        return fail(PH_EINVAL, "coef_limbs must be 1, 2 or 4");
    if (eq_term_off[0] != 0) return fail(PH_EINVAL, "eq_term_off[0] must be 0");
    for (int i = 0; i < n_eq; ++i)
        if (eq_term_off[i + 1] < eq_term_off[i]) return fail(PH_EINVAL, "eq_term_off not monotone");
    int64_t T = eq_term_off[n_eq];
    if (term_fac_off[0] != 0) return fail(PH_EINVAL, "term_fac_off[0] must be 0");
    for (int64_t t = 0; t < T; ++t) {
        int a = term_fac_off[t], b = term_fac_off[t + 1];
        if (b < a) return fail(PH_EINVAL, "term_fac_off not monotone");
        if (b - a > 32) return fail(PH_EUNSUPPORTED, "a term has more than 32 factors");
        for (int q = a; q < b; ++q) {
            if (!fac_var || !fac_exp) return fail(PH_EINVAL, "null factor array");
            if (fac_var[q] < 0 || fac_var[q] >= n_var)
                return fail(PH_EINVAL, "factor variable out of range");
            if (q > a && fac_var[q] <= fac_var[q - 1])
                return fail(PH_EINVAL, "factor variables must strictly increase within a term");
            if (fac_exp[q] < 1 || fac_exp[q] > 64)
                return fail(PH_EINVAL, "factor exponent must be in 1..64");
        }
    }
    return PH_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int ph_system_create(int32_t n_eq, int32_t n_var, const int32_t *eq_term_off,
                                const int32_t *term_fac_off, const int32_t *fac_var,
                                const int32_t *fac_exp, const double *coef, int32_t coef_limbs,
                                ph_system **out)
{
    if (!out) return fail(PH_EINVAL, "out is null");
    *out = nullptr;
    int rc = validate(n_eq, n_var, eq_term_off, term_fac_off, fac_var, fac_exp, coef, coef_limbs);
    if (rc) return rc;
    std::unique_ptr<ph_system> s(new ph_system());
    HostSystem &h = s->h;
    h.n_eq = n_eq;
    h.n_var = n_var;
    int64_t T = eq_term_off[n_eq];
    int64_t F = term_fac_off[T];
    h.eq_term_off.assign(eq_term_off, eq_term_off + n_eq + 1);
    h.term_fac_off.assign(term_fac_off, term_fac_off + T + 1);
    if (F > 0) {
        h.fac_var.assign(fac_var, fac_var + F);
        h.fac_exp.assign(fac_exp, fac_exp + F);
    }
    h.coef.assign(size_t(T) * 8, 0.0);
    for (int64_t t = 0; t < T; ++t)
        for (int c = 0; c < 2; ++c)
            for (int l = 0; l < coef_limbs; ++l)
                h.coef[size_t(t) * 8 + c * 4 + l] = coef[(size_t(t) * 2 + c) * coef_limbs + l];
    h.deg.assign(n_eq, 0);
    for (int i = 0; i < n_eq; ++i) {
        int best = 0;
        for (int t = eq_term_off[i]; t < eq_term_off[i + 1]; ++t) {
            int d = 0;
            for (int q = term_fac_off[t]; q < term_fac_off[t + 1]; ++q) d += fac_exp[q];
            best = std::max(best, d);
            h.max_k = std::max(h.max_k, term_fac_off[t + 1] - term_fac_off[t]);
        }
        h.deg[i] = best;
    }
    // FNV-1a fingerprint of the defining arrays (autotuning cache key)
    uint64_t fp = 1469598103934665603ull;
    auto mix = [&fp](const void *p, size_t nb) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < nb; ++i) fp = (fp ^ b[i]) * 1099511628211ull;
    };
    mix(&n_eq, sizeof n_eq);
    mix(&n_var, sizeof n_var);
    mix(h.eq_term_off.data(), h.eq_term_off.size() * 4);
    mix(h.term_fac_off.data(), h.term_fac_off.size() * 4);
    if (F > 0) {
        mix(h.fac_var.data(), h.fac_var.size() * 4);
        mix(h.fac_exp.data(), h.fac_exp.size() * 4);
    }
    mix(h.coef.data(), h.coef.size() * 8);
    h.fingerprint = fp;
    PH_HIP(hipGetDevice(&s->device));
    rc = build_table(h, nullptr, s->total);
    if (rc) return rc;
    load_eval_cache(s.get());
    *out = s.release();
    return PH_OK;
}

extern "C" int ph_system_destroy(ph_system *s)
{
    if (!s) return fail(PH_EINVAL, "null system");
    (void)hipDeviceSynchronize();
    free_table(s->total);
    for (auto &kv : s->with_start) free_table(kv.second);
    delete s;
    return PH_OK;
}

extern "C" int ph_system_info(const ph_system *s, int32_t *n_eq, int32_t *n_var, int64_t *n_terms,
                              int32_t *max_factors)
{
    if (!s) return fail(PH_EINVAL, "null system");
    if (n_eq) *n_eq = s->h.n_eq;
    if (n_var) *n_var = s->h.n_var;
    if (n_terms) *n_terms = s->h.eq_term_off.back();
    if (max_factors) *max_factors = s->h.max_k;
    return PH_OK;
}

extern "C" int ph_system_degrees(const ph_system *s, int32_t *deg)
{
    if (!s || !deg) return fail(PH_EINVAL, "null argument");
    for (int i = 0; i < s->h.n_eq; ++i) deg[i] = s->h.deg[i];
    return PH_OK;
}

extern "C" const char *ph_last_error(void) { return g_err.c_str(); }

extern "C" int ph_track_opts_default(ph_track_opts *o)
{
    if (!o) return fail(PH_EINVAL, "null opts");
    o->prec = PH_D;
    o->mixed = 0;
    o->predictor_order = 1;
    o->max_newton = 3;
    o->expand_after = 3;
    o->polish_max = 8;
    o->h_init = 0.01;
    o->h_min = 1e-10;
    o->h_max = 0.1;
    o->shrink = 0.5;
    o->expand = 1.5;
    o->tol_dx = 1e-8;
    o->diverge_norm = 1e8;
    o->polish_tol = -1.0;
    o->max_steps = 100000;
    o->schedule = PH_SCHED_PERSISTENT;
    o->rounds_per_launch = 32;
    o->launches_per_sync = 8;
    o->blocks_per_cu = 0;
    o->lanes_per_path = 0;
    o->tol_res = 1e-6;
    o->launch_ms = 2.0;
    return PH_OK;
}
