// Parameter choice (include/hdc_tune.h): the experience-based autotuner of
// section 4 (A0, the exhaustive search of section 4.2, separable per axis for
// N-D problems; A1, the experience of section 4.3) over a JSON-lines timing
// database (section 5.1), and inference of the learned predictor of section
// 4.4 through the MLP kernels of hdc_mlp.h.  Only the public C ABI of the
// library is used here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <ctime>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/hdc.h"
#include "../../include/hdc_mlp.h"
#include "../../include/hdc_tune.h"
#include "hdc_internal.h"

namespace {

hdc_status fail(hdc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(st, buf);
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t _e = (expr);                                                           \
        if (_e != hipSuccess) return fail(HDC_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

constexpr int kPClasses[8] = {1, 2, 3, 4, 6, 8, 12, 16};
constexpr int64_t kMaxM = int64_t(1) << 22;       // 1D and innermost axes
constexpr int64_t kMaxOuterM = int64_t(1) << 20;  // outer N-D axes (two column stages)

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
int64_t pow2_ceil(int64_t x) {
    int64_t v = 1;
    while (v < x) v <<= 1;
    return v;
}
bool in_pclasses(int64_t p) {
    for (int c : kPClasses)
        if (c == p) return true;
    return false;
}

// ----------------------------------------------------------- tiny JSON --
// Enough of JSON for the database rows: objects, arrays, strings, numbers,
// true / false / null.
struct JVal {
    enum Kind { NUL, NUM, STR, ARR, OBJ, BOOL } kind = NUL;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const char* k) const {
        for (auto& kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    static constexpr int kMaxDepth = 64;  // nesting limit: a malformed line cannot exhaust the stack
    const char* s;
    const char* e;
    bool ok = true;
    int depth = 0;
    void ws() {
        while (s < e && std::isspace((unsigned char)*s)) ++s;
    }
    bool lit(const char* w) {
        size_t n = strlen(w);
        if ((size_t)(e - s) >= n && !strncmp(s, w, n)) {
            s += n;
            return true;
        }
        return false;
    }
    std::string string() {
        std::string out;
        if (s >= e || *s != '"') {
            ok = false;
            return out;
        }
        ++s;
        while (s < e && *s != '"') {
            char c = *s++;
            if (c == '\\' && s < e) {
                char x = *s++;
                switch (x) {
                    case 'n': out += '\n'; break;
                    case 't': out += '\t'; break;
                    case 'r': out += '\r'; break;
                    case 'b': out += '\b'; break;
                    case 'f': out += '\f'; break;
                    case 'u': {
                        if (e - s < 4) {
                            ok = false;
                            return out;
                        }
                        unsigned v = (unsigned)strtoul(std::string(s, 4).c_str(), nullptr, 16);
                        s += 4;
                        out += v < 128 ? (char)v : '?';
                        break;
                    }
                    default: out += x;
                }
            } else {
                out += c;
            }
        }
        if (s >= e) {
            ok = false;
            return out;
        }
        ++s;
        return out;
    }
    JVal value() {
        JVal v;
        if (depth >= kMaxDepth) {
            ok = false;
            return v;
        }
        struct Nest {
            int& d;
            explicit Nest(int& x) : d(x) { ++d; }
            ~Nest() { --d; }
        } nest(depth);
        ws();
        if (s >= e) {
            ok = false;
            return v;
        }
        if (*s == '{') {
            ++s;
            v.kind = JVal::OBJ;
            ws();
            if (s < e && *s == '}') {
                ++s;
                return v;
            }
            while (ok) {
                ws();
                std::string k = string();
                ws();
                if (s >= e || *s != ':') {
                    ok = false;
                    break;
                }
                ++s;
                JVal x = value();
                v.obj.emplace_back(k, x);
                ws();
                if (s < e && *s == ',') {
                    ++s;
                    continue;
                }
                if (s < e && *s == '}') {
                    ++s;
                    break;
                }
                ok = false;
            }
        } else if (*s == '[') {
            ++s;
            v.kind = JVal::ARR;
            ws();
            if (s < e && *s == ']') {
                ++s;
                return v;
            }
            while (ok) {
                v.arr.push_back(value());
                ws();
                if (s < e && *s == ',') {
                    ++s;
                    continue;
                }
                if (s < e && *s == ']') {
                    ++s;
                    break;
                }
                ok = false;
            }
        } else if (*s == '"') {
            v.kind = JVal::STR;
            v.str = string();
        } else if (lit("true")) {
            v.kind = JVal::BOOL;
            v.num = 1;
        } else if (lit("false")) {
            v.kind = JVal::BOOL;
        } else if (lit("null")) {
            v.kind = JVal::NUL;
        } else {
            char* end = nullptr;
            v.num = strtod(s, &end);
            if (end == s) ok = false;
            s = end;
            v.kind = JVal::NUM;
        }
        return v;
    }
};

std::string jstr(const std::string& x) {
    std::string o = "\"";
    for (char c : x) {
        if (c == '"' || c == '\\') {
            o += '\\';
            o += c;
        } else if ((unsigned char)c < 0x20) {
            char b[8];
            snprintf(b, sizeof b, "\\u%04x", (unsigned)c);
            o += b;
        } else {
            o += c;
        }
    }
    return o + "\"";
}

// ------------------------------------------------------------ database --

// One candidate: per axis (m, D, tile); p and q follow from m.
struct Cand {
    int64_t m[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    int32_t tile[3] = {0, 0, 0};
    bool operator==(const Cand& o) const {
        for (int a = 0; a < 3; ++a)
            if (m[a] != o.m[a] || D[a] != o.D[a] || tile[a] != o.tile[a]) return false;
        return true;
    }
};

const char* dtype_name(hdc_dtype t) { return t == HDC_C128 ? "c128" : "c64"; }

// The problem key, as the Python binding writes it (json.dumps with sorted keys).
std::string problem_key(const hdc_problem& pr) {
    std::string L = "[", M = "[";
    for (int a = 0; a < pr.ndim; ++a) {
        L += (a ? ", " : "") + std::to_string(pr.L[a]);
        M += (a ? ", " : "") + std::to_string(pr.M[a]);
    }
    return "{\"L\": " + L + "], \"M\": " + M + "], \"batch\": " + std::to_string(pr.batch) + ", \"dtype\": \"" +
           dtype_name(pr.dtype) + "\"}";
}

std::string params_json(const Cand& c, int nd) {
    auto list = [&](auto get) {
        std::string o = "[";
        for (int a = 0; a < nd; ++a) o += (a ? ", " : "") + std::to_string((long long)get(a));
        return o + "]";
    };
    bool tiled = false;
    for (int a = 0; a < nd; ++a) tiled |= c.tile[a] != 0;
    std::string o;
    if (nd == 1) {
        o = "{\"D\": " + std::to_string(c.D[0]) + ", \"m\": " + std::to_string(c.m[0]);
        if (tiled) o += ", \"tile\": " + std::to_string(c.tile[0]);
    } else {
        o = "{\"D\": " + list([&](int a) { return c.D[a]; }) + ", \"m\": " + list([&](int a) { return c.m[a]; });
        if (tiled) o += ", \"tile\": " + list([&](int a) { return (int64_t)c.tile[a]; });
    }
    return o + "}";
}

bool cand_from_json(const JVal& p, int nd, Cand* c) {
    const JVal* m = p.get("m");
    const JVal* D = p.get("D");
    const JVal* t = p.get("tile");
    if (!m || !D) return false;
    *c = Cand{};
    for (int a = 0; a < nd; ++a) {
        auto at = [&](const JVal* v) -> double {
            if (v->kind == JVal::NUM) return a == 0 ? v->num : -1;
            if (v->kind == JVal::ARR && (int)v->arr.size() > a && v->arr[a].kind == JVal::NUM) return v->arr[a].num;
            return -1;
        };
        const double mv = at(m), dv = at(D), tv = t ? at(t) : 0;
        // integral values within range before any conversion
        auto whole = [](double x, double lo, double hi) { return x >= lo && x <= hi && x == std::floor(x); };
        if (!whole(mv, 1, 1099511627776.0) || !whole(dv, 1, 1099511627776.0) || !whole(tv, 0, 65536)) return false;
        c->m[a] = (int64_t)mv;
        c->D[a] = (int64_t)dv;
        c->tile[a] = (int32_t)tv;
    }
    return true;
}

struct Row {
    std::string key;
    Cand c;
    double ms;
};

struct DB {
    std::string path, device, build;
    std::vector<Row> rows;  // rows of this device and build only
    void load() {
        rows.clear();
        if (path.empty()) return;
        FILE* fh = fopen(path.c_str(), "r");
        if (!fh) return;
        std::string line;
        char buf[4096];
        while (fgets(buf, sizeof buf, fh)) {
            line += buf;
            if (line.empty() || line.back() != '\n') continue;
            parse(line);
            line.clear();
        }
        if (!line.empty()) parse(line);  // a final line without newline
        fclose(fh);
    }
    void parse(const std::string& line) {
        JParser P{line.data(), line.data() + line.size()};
        JVal v = P.value();
        if (!P.ok || v.kind != JVal::OBJ) return;  // e.g. a line cut short by a kill
        const JVal *k = v.get("key"), *p = v.get("params"), *ms = v.get("ms"), *dv = v.get("device"),
                   *bd = v.get("build");
        if (!k || !p || !ms || !dv || !bd || k->kind != JVal::STR || ms->kind != JVal::NUM) return;
        if (dv->str != device || bd->str != build) return;
        JParser KP{k->str.data(), k->str.data() + k->str.size()};
        JVal kv = KP.value();
        const JVal* L = kv.get("L");
        const int nd = (L && L->kind == JVal::ARR) ? (int)L->arr.size() : 1;
        Row r;
        r.key = k->str;
        r.ms = ms->num;
        if (nd < 1 || nd > 3 || !cand_from_json(*p, nd, &r.c)) return;
        rows.push_back(r);
    }
    void add(const std::string& key, const Cand& c, int nd, double ms) {
        rows.push_back({key, c, ms});
        if (path.empty()) return;
        FILE* fh = fopen(path.c_str(), "a+");
        if (!fh) return;
        // a record cut short by a kill leaves no newline: start a fresh line
        if (fseek(fh, -1, SEEK_END) == 0) {
            const int last = fgetc(fh);
            if (last != '\n' && last != EOF) fputc('\n', fh);
        }
        fseek(fh, 0, SEEK_END);
        fprintf(fh, "{\"key\": %s, \"params\": %s, \"ms\": %.9g, \"device\": %s, \"build\": %s, \"t\": %lld}\n",
                jstr(key).c_str(), params_json(c, nd).c_str(), ms, jstr(device).c_str(), jstr(build).c_str(),
                (long long)time(nullptr));
        fclose(fh);
    }
};

// -------------------------------------------------------------- search --

using CostFn = std::function<double(const hdc_params&)>;

hdc_params to_params(const Cand& c) {
    hdc_params p{};
    for (int a = 0; a < 3; ++a) {
        p.m[a] = c.m[a];
        p.D[a] = c.D[a];
        p.tile[a] = c.tile[a];
    }
    return p;
}

int64_t axis_limit(const hdc_problem& pr, int a) { return (pr.ndim > 1 && a < pr.ndim - 1) ? kMaxOuterM : kMaxM; }

// The m of a scale-free class p on axis a: the smallest power of two with
// ceil(L/m) <= p, at most the axis limit, doubled while q < p.
int64_t m_for_class(const hdc_problem& pr, int a, int64_t p) {
    const int64_t L = pr.L[a], M = pr.M[a];
    int64_t m = pow2_ceil(cdiv(L, p));
    while (m > axis_limit(pr, a)) m /= 2;
    while (cdiv(M, m) < cdiv(L, m)) m *= 2;
    return m;
}

Cand default_cand(const hdc_problem& pr) {
    Cand c;
    for (int a = 0; a < pr.ndim; ++a) {
        c.m[a] = m_for_class(pr, a, 1);
        c.D[a] = cdiv(std::max(pr.M[a], 2 * pr.L[a] - 1), c.m[a]);
    }
    return c;
}

// (m, D) candidates of one axis (section 4.2's grid): power-of-two m with
// p = ceil(L/m) in the classes (or q = 1) and q >= p; D = q, and with
// all_d also 1, 2, 4, ... < q.
// 1D problems also take m = R 2^k with R in these odd 7-smooth factors (the
// mixed-radix fused kernel; such m only fit the fused kernel, m <= 4096)
constexpr int kOddR[] = {3, 5, 7, 9, 15, 21, 25, 27, 35, 45, 49, 63};

std::vector<std::pair<int64_t, int64_t>> axis_grid(const hdc_problem& pr, int a, bool all_d) {
    std::vector<std::pair<int64_t, int64_t>> out;
    const int64_t L = pr.L[a], K = std::max(pr.M[a], 2 * pr.L[a] - 1);
    std::vector<int64_t> ms;
    for (int64_t m = 1; m <= axis_limit(pr, a); m *= 2) ms.push_back(m);
    if (pr.ndim == 1)
        for (int R : kOddR)
            for (int64_t m = R; m <= 4096; m *= 2) ms.push_back(m);
    std::sort(ms.begin(), ms.end());
    for (int64_t m : ms) {
        const int64_t p = cdiv(L, m), q = cdiv(K, m);
        if (q < p || !(in_pclasses(p) || q == 1)) continue;
        out.push_back({m, q});
        // D only sizes the workspace of the column/row passes: the fused kernel
        // (every m = R 2^k) runs the same for any D
        if (all_d && (m & (m - 1)) == 0)
            for (int64_t d = 1; d < q; d *= 2) out.push_back({m, d});
    }
    return out;
}

struct Search {
    const hdc_problem& pr;
    DB& db;
    CostFn cost;
    std::string key;
    std::vector<std::pair<Cand, double>> table;  // timings of this search (and reused rows)
    hdc_status err = HDC_OK;

    Search(const hdc_problem& p, DB& d, CostFn c) : pr(p), db(d), cost(std::move(c)), key(problem_key(p)) {}

    bool admissible(const Cand& c) {
        hdc_params p = to_params(c);
        return hdc_params_check(&pr, &p, nullptr) == HDC_OK;
    }
    const double* known(const Cand& c) {
        for (auto& t : table)
            if (t.first == c) return &t.second;
        return nullptr;
    }
    // time candidate c (once per search); returns its ms or a negative value
    double run(const Cand& c) {
        if (const double* k = known(c)) return *k;
        if (!admissible(c)) return -1;
        const double ms = cost(to_params(c));
        if (!(ms >= 0)) return -1;
        table.push_back({c, ms});
        db.add(key, c, pr.ndim, ms);
        return ms;
    }
    // argmin with the tie rule: within 1 %, the smaller m (axis by axis), then
    // the smaller D, then the default tile, then the smaller tile
    bool pick(Cand* best, double* best_ms) const {
        if (table.empty()) return false;
        double lo = table[0].second;
        for (auto& t : table) lo = std::min(lo, t.second);
        const std::pair<Cand, double>* w = nullptr;
        auto key = [&](const Cand& c) {
            std::vector<int64_t> k;
            for (int a = 0; a < pr.ndim; ++a) k.push_back(c.m[a]);
            for (int a = 0; a < pr.ndim; ++a) k.push_back(c.D[a]);
            for (int a = 0; a < pr.ndim; ++a) k.push_back(c.tile[a] == 0 ? 0 : 1 + c.tile[a]);
            return k;
        };
        for (auto& t : table) {
            if (t.second > lo * 1.01) continue;
            if (!w || key(t.first) < key(w->first) || (key(t.first) == key(w->first) && t.second < w->second))
                w = &t;
        }
        *best = w->first;
        *best_ms = w->second;
        return true;
    }
    // column tiles of the best: half and double the default on every axis that
    // runs column passes, one axis at a time
    void tiles(const Cand& base) {
        for (int a = 0; a < pr.ndim; ++a) {
            hdc_params in = to_params(base), out{};
            in.tile[a] = 0;
            if (hdc_params_check(&pr, &in, &out) != HDC_OK || out.tile[a] == 0) continue;
            for (int t : {out.tile[a] / 2, out.tile[a] * 2}) {
                if (t < 1) continue;
                Cand c = base;
                c.tile[a] = t;
                run(c);
            }
        }
    }

    // A0: the whole grid (1D); per axis with the others at their defaults (N-D)
    void a0() {
        if (pr.ndim == 1) {
            for (auto& md : axis_grid(pr, 0, true)) {
                Cand c;
                c.m[0] = md.first;
                c.D[0] = md.second;
                run(c);
            }
        } else {
            const Cand base = default_cand(pr);
            Cand comb = base;
            for (int a = 0; a < pr.ndim; ++a) {
                double best = -1;
                for (auto& md : axis_grid(pr, a, true)) {
                    Cand c = base;
                    c.m[a] = md.first;
                    c.D[a] = md.second;
                    const double t = run(c);
                    if (t >= 0 && (best < 0 || t < best * 0.99)) {
                        best = t;
                        comb.m[a] = md.first;
                        comb.D[a] = md.second;
                    }
                }
            }
            // the combination of the per-axis bests is what A0 returns for N-D
            // (section 4.2's separability), with its column tiles
            run(comb);
            comb_ = comb;
            has_comb_ = true;
            tiles(comb);
            return;
        }
        Cand b;
        double bms;
        if (pick(&b, &bms)) tiles(b);
    }
    Cand comb_;
    bool has_comb_ = false;

    bool final_pick(Cand* best, double* best_ms) const {
        if (!has_comb_) return pick(best, best_ms);
        // among the combination and its tile variants (same m and D)
        Search tmp(pr, db, cost);
        for (auto& t : table) {
            bool same = true;
            for (int a = 0; a < pr.ndim; ++a) same &= t.first.m[a] == comb_.m[a] && t.first.D[a] == comb_.D[a];
            if (same) tmp.table.push_back(t);
        }
        return tmp.pick(best, best_ms);
    }

    // classes (p, D-mode) per axis of the best entries of the two nearest tuned
    // problems of this dtype and dimension
    std::vector<Cand> experience() {
        struct K {
            double dist;
            Cand c;
        };
        std::map<std::string, std::pair<Cand, double>> bests;
        std::map<std::string, hdc_problem> probs;
        for (auto& r : db.rows) {
            if (r.key == key) continue;
            JParser P{r.key.data(), r.key.data() + r.key.size()};
            JVal v = P.value();
            const JVal *L = v.get("L"), *M = v.get("M"), *dt = v.get("dtype"), *bt = v.get("batch");
            if (!P.ok || !L || !M || !dt || L->kind != JVal::ARR || (int)L->arr.size() != pr.ndim) continue;
            if (dt->str != dtype_name(pr.dtype)) continue;
            hdc_problem q{};
            q.ndim = pr.ndim;
            q.dtype = pr.dtype;
            q.batch = bt ? (int64_t)bt->num : 1;
            for (int a = 0; a < pr.ndim; ++a) {
                q.L[a] = (int64_t)L->arr[a].num;
                q.M[a] = (int64_t)M->arr[a].num;
            }
            probs[r.key] = q;
            auto it = bests.find(r.key);
            if (it == bests.end() || r.ms < it->second.second) bests[r.key] = {r.c, r.ms};
        }
        std::vector<K> ks;
        for (auto& b : bests) {
            const hdc_problem& q = probs[b.first];
            double dist = 0;
            for (int a = 0; a < pr.ndim; ++a) dist += std::fabs(std::log2((double)q.L[a]) - std::log2((double)pr.L[a]));
            // the class of its best on each axis, mapped onto this problem
            Cand c;
            for (int a = 0; a < pr.ndim; ++a) {
                const int64_t p = cdiv(q.L[a], b.second.first.m[a]);
                const int64_t qq = cdiv(std::max(q.M[a], 2 * q.L[a] - 1), b.second.first.m[a]);
                int64_t pc = kPClasses[0];
                for (int x : kPClasses)
                    if (std::fabs(std::log2((double)x) - std::log2((double)p)) <
                        std::fabs(std::log2((double)pc) - std::log2((double)p)))
                        pc = x;
                c.m[a] = m_for_class(pr, a, pc);
                const int64_t qn = cdiv(std::max(pr.M[a], 2 * pr.L[a] - 1), c.m[a]);
                c.D[a] = b.second.first.D[a] >= qq ? qn : std::min<int64_t>(b.second.first.D[a], qn);
            }
            ks.push_back({dist, c});
        }
        std::stable_sort(ks.begin(), ks.end(), [](const K& x, const K& y) { return x.dist < y.dist; });
        std::vector<Cand> out;
        for (auto& k : ks) {
            if (std::find(out.begin(), out.end(), k.c) == out.end()) out.push_back(k.c);
            if (out.size() >= 2) break;
        }
        return out;
    }

    // A1: database reuse, experience, random candidates, local refinement
    bool a1(bool* reused) {
        *reused = false;
        for (auto& r : db.rows)
            if (r.key == key) table.push_back({r.c, r.ms});
        if (!table.empty()) {
            *reused = true;
            return true;
        }
        std::vector<Cand> seeds = experience();
        seeds.push_back(default_cand(pr));
        for (auto& c : seeds) run(c);
        // random candidates: axis and (m, D = q) drawn by a seeded generator
        uint64_t st = 0x9e3779b97f4a7c15ull;
        for (char ch : key) st = (st ^ (uint64_t)(unsigned char)ch) * 0x100000001b3ull;
        auto rnd = [&]() {
            st += 0x9e3779b97f4a7c15ull;
            uint64_t z = st;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            return z ^ (z >> 31);
        };
        Cand cur;
        double cur_ms;
        for (int i = 0; i < 2; ++i) {
            if (!pick(&cur, &cur_ms)) cur = default_cand(pr);
            const int a = (int)(rnd() % (uint64_t)pr.ndim);
            auto grid = axis_grid(pr, a, false);
            std::vector<Cand> fresh;
            for (auto& md : grid) {
                Cand c = cur;
                c.m[a] = md.first;
                c.D[a] = md.second;
                c.tile[a] = 0;
                if (!known(c) && admissible(c)) fresh.push_back(c);
            }
            if (!fresh.empty()) run(fresh[rnd() % fresh.size()]);
        }
        // local refinement around the incumbent
        for (int round = 0; round < 3; ++round) {
            if (!pick(&cur, &cur_ms)) break;
            const size_t before = table.size();
            for (int a = 0; a < pr.ndim; ++a) {
                for (int64_t m : {cur.m[a] / 2, cur.m[a] * 2}) {
                    if (m < 1 || m > axis_limit(pr, a)) continue;
                    Cand c = cur;
                    c.m[a] = m;
                    c.D[a] = cdiv(std::max(pr.M[a], 2 * pr.L[a] - 1), m);
                    c.tile[a] = 0;
                    run(c);
                }
                const int64_t q = cdiv(std::max(pr.M[a], 2 * pr.L[a] - 1), cur.m[a]);
                if (cur.D[a] < q) {
                    Cand c = cur;
                    c.D[a] = q;
                    run(c);
                }
            }
            if (table.size() == before) break;
        }
        return !table.empty();
    }
};

hdc_status tune_core(const hdc_problem* pr, int mode, DB& db, CostFn cost, hdc_params* best, double* best_ms) {
    if (!pr || !best) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    if (mode != 0 && mode != 1) return fail(HDC_ERR_INVALID_ARG, "mode %d: 0 (A0) or 1 (A1)", mode);
    {
        hdc_params d = to_params(default_cand(*pr));
        hdc_status st = hdc_params_check(pr, &d, nullptr);
        if (st != HDC_OK) return st;
    }
    db.load();
    Search S(*pr, db, std::move(cost));
    Cand b;
    double bms = 0;
    if (mode == 0) {
        S.a0();
        if (!S.final_pick(&b, &bms)) return fail(HDC_ERR_UNSUPPORTED, "no candidate could be timed");
    } else {
        bool reused = false;
        if (!S.a1(&reused) || !S.pick(&b, &bms)) return fail(HDC_ERR_UNSUPPORTED, "no candidate could be timed");
    }
    hdc_params in = to_params(b), out{};
    hdc_status st = hdc_params_check(pr, &in, &out);
    if (st != HDC_OK) return st;
    // report the tile as chosen (0 = default), with p, q, D and C derived
    for (int a = 0; a < 3; ++a) out.tile[a] = b.tile[a];
    *best = out;
    if (best_ms) *best_ms = bms;
    return HDC_OK;
}

// ----------------------------------------------------------- GPU timing --

template <typename T>
__global__ void k_fill_uniform(T* x, int64_t n, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + (uint64_t)i * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    x[i] = (T)((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
}

struct GpuTimer {
    hipStream_t s = nullptr;
    void *f = nullptr, *g = nullptr, *h = nullptr, *ws = nullptr;
    size_t ws_cap = 0;
    ~GpuTimer() {
        if (s) (void)hipStreamSynchronize(s);
        for (void* p : {f, g, h, ws})
            if (p) (void)hipFree(p);
        if (s) (void)hipStreamDestroy(s);
    }
    hdc_status init(const hdc_problem& pr) {
        HIP_TRY(hipStreamCreate(&s));
        int64_t nin = pr.batch, nout = pr.batch;
        for (int a = 0; a < pr.ndim; ++a) {
            nin *= pr.L[a];
            nout *= pr.M[a];
        }
        const size_t b = pr.dtype == HDC_C128 ? 16 : 8;
        HIP_TRY(hipMalloc(&f, (size_t)nin * b));
        HIP_TRY(hipMalloc(&g, (size_t)nin * b));
        HIP_TRY(hipMalloc(&h, (size_t)nout * b));
        const int64_t nr = 2 * nin;  // real scalars
        const unsigned blocks = (unsigned)((nr + 255) / 256);
        if (pr.dtype == HDC_C128) {
            hipLaunchKernelGGL(k_fill_uniform<double>, dim3(blocks), dim3(256), 0, s, (double*)f, nr, 1ull);
            hipLaunchKernelGGL(k_fill_uniform<double>, dim3(blocks), dim3(256), 0, s, (double*)g, nr, 2ull);
        } else {
            hipLaunchKernelGGL(k_fill_uniform<float>, dim3(blocks), dim3(256), 0, s, (float*)f, nr, 1ull);
            hipLaunchKernelGGL(k_fill_uniform<float>, dim3(blocks), dim3(256), 0, s, (float*)g, nr, 2ull);
        }
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s));
        return HDC_OK;
    }
    // median of 5 timed runs after 2 warm-ups; negative for a set that cannot run
    double time(const hdc_problem& pr, const hdc_params& pm) {
        hdc_plan_t P = nullptr;
        if (hdc_plan_params(&P, &pr, &pm) != HDC_OK) return -1;
        size_t need = 0;
        (void)hdc_workspace_size(P, &need);
        if (need > ws_cap) {
            (void)hipStreamSynchronize(s);
            if (ws) (void)hipFree(ws);
            ws = nullptr;
            ws_cap = 0;
            if (hipMalloc(&ws, need) != hipSuccess) {
                ws = nullptr;
                hdc_plan_destroy(P);
                return -1;
            }
            ws_cap = need;
        }
        float ms[5];
        const hdc_status st = hdc_time_convolve(P, f, g, h, need ? ws : nullptr, s, 2, 5, ms);
        hdc_plan_destroy(P);
        if (st != HDC_OK) return -1;
        std::sort(ms, ms + 5);
        return ms[2];
    }
};

std::string device_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    return prop.name;
}

// ------------------------------------------------------------ predictor --

constexpr int kFeatures = 12;
constexpr int kClasses = 16;         // (p, D-mode) classes
constexpr int kMaxClasses = 17;      // ... and explicit padding (q = 1)
// features outside the training range by more than this (1/16 of an octave in
// the scaled length features) make an axis abstain
constexpr float kRangeMargin = 1.0f / 16.0f;

void features(const hdc_problem& pr, int axis, float* v) {
    const int nd = pr.ndim;
    double others[2] = {1, 1};
    int k = 0;
    for (int a = 0; a < nd; ++a)
        if (a != axis) others[k++] = (double)pr.L[a];
    v[0] = (float)(std::log2((double)pr.L[axis]) / 16.0);
    v[1] = (float)(std::log2(others[0]) / 16.0);
    v[2] = (float)(std::log2(others[1]) / 16.0);
    for (int a = 0; a < 3; ++a) v[3 + a] = axis == a ? 1.f : 0.f;
    for (int d = 1; d <= 3; ++d) v[5 + d] = nd == d ? 1.f : 0.f;
    v[9] = pr.dtype == HDC_C128 ? 1.f : 0.f;
    const double batch = (double)std::max<int64_t>(pr.batch, 1);
    v[10] = (float)(std::log2(batch) / 16.0);
    double n = batch;
    for (int a = 0; a < nd; ++a) n *= (double)pr.L[a];
    v[11] = (float)(std::log2(std::max(1.0, n)) / 32.0);
}

// --------------------------------------------------------- batch buckets --

// Key of an uneven batch's bucket: the problems whose next power of two of L is
// `size` (the grouping of the per-bucket search).
std::string bucket_key(int64_t size, hdc_dtype dt) {
    return "{\"bucket\": " + std::to_string((long long)size) + ", \"dtype\": \"" + dtype_name(dt) + "\"}";
}

// Fastest recorded m per bucket size (rows of `device` and `build` only; equal
// times go to the larger m): size -> (ms, m).
std::map<int64_t, std::pair<double, int64_t>> bucket_best(const char* path, hdc_dtype dt, const std::string& device,
                                                          const std::string& build) {
    std::map<int64_t, std::pair<double, int64_t>> best;
    FILE* fh = fopen(path, "r");
    if (!fh) return best;
    auto take = [&](const std::string& line) {
        JParser P{line.data(), line.data() + line.size()};
        JVal v = P.value();
        if (!P.ok || v.kind != JVal::OBJ) return;
        const JVal *k = v.get("key"), *p = v.get("params"), *ms = v.get("ms"), *dv = v.get("device"),
                   *bd = v.get("build");
        if (!k || !p || !ms || !dv || !bd || k->kind != JVal::STR || ms->kind != JVal::NUM ||
            dv->kind != JVal::STR || bd->kind != JVal::STR || p->kind != JVal::OBJ)
            return;
        if (dv->str != device || bd->str != build) return;
        JParser KP{k->str.data(), k->str.data() + k->str.size()};
        JVal kv = KP.value();
        if (!KP.ok || kv.kind != JVal::OBJ) return;
        const JVal *sz = kv.get("bucket"), *dt_s = kv.get("dtype"), *m = p->get("m");
        if (!sz || !dt_s || !m || sz->kind != JVal::NUM || dt_s->kind != JVal::STR || m->kind != JVal::NUM) return;
        // integral sizes within range before any conversion (an FFT size above the
        // library's largest m, or a bucket beyond 2^40, is not a row of this kind)
        if (dt_s->str != dtype_name(dt) || !(ms->num >= 0)) return;
        if (!(sz->num >= 1 && sz->num <= 1099511627776.0 && sz->num == std::floor(sz->num))) return;
        if (!(m->num >= 1 && m->num <= (double)kMaxM && m->num == std::floor(m->num))) return;
        const int64_t size = (int64_t)sz->num, mm = (int64_t)m->num;
        auto it = best.find(size);
        if (it == best.end() || ms->num < it->second.first || (ms->num == it->second.first && mm > it->second.second))
            best[size] = {ms->num, mm};
    };
    std::string line;
    char buf[4096];
    while (fgets(buf, sizeof buf, fh)) {
        line += buf;
        if (line.empty() || line.back() != '\n') continue;
        take(line);
        line.clear();
    }
    if (!line.empty()) take(line);
    fclose(fh);
    return best;
}

}  // namespace

struct hdc_predictor_s {
    std::vector<int> sizes;
    bool ranged = false;           // format 2: the training range is known
    float lo[kFeatures], hi[kFeatures];
    std::vector<float*> W, b;  // device
    float *x = nullptr, *y0 = nullptr, *y1 = nullptr, *P = nullptr;
    hipStream_t s = nullptr;
    ~hdc_predictor_s() {
        for (float* p : W) (void)hipFree(p);
        for (float* p : b) (void)hipFree(p);
        for (float* p : {x, y0, y1, P})
            if (p) (void)hipFree(p);
        if (s) (void)hipStreamDestroy(s);
    }
};

extern "C" {

const char* hdc_build_id(void) { return "hdc 0.1 (gfx950) built " __DATE__ " " __TIME__; }

hdc_status hdc_tune(const hdc_problem* prob, int mode, const char* db, hdc_params* best, double* best_ms) {
    if (!prob || !best) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    DB d;
    d.path = db ? db : "";
    d.device = device_name();
    d.build = hdc_build_id();
    GpuTimer T;
    {
        hdc_params dflt = to_params(default_cand(*prob));
        hdc_status st = hdc_params_check(prob, &dflt, nullptr);
        if (st != HDC_OK) return st;
    }
    hdc_status st = T.init(*prob);
    if (st != HDC_OK) return st;
    const hdc_problem pr = *prob;
    return tune_core(prob, mode, d, [&](const hdc_params& pm) { return T.time(pr, pm); }, best, best_ms);
}

hdc_status hdc_tune_host(const hdc_problem* prob, int mode, const char* db, const char* device, const char* build,
                         hdc_cost_fn cost, void* ctx, hdc_params* best, double* best_ms) {
    if (!prob || !best || !cost || !device || !build) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    DB d;
    d.path = db ? db : "";
    d.device = device;
    d.build = build;
    const hdc_problem pr = *prob;
    return tune_core(prob, mode, d,
                     [&](const hdc_params& pm) {
                         hdc_params full{};
                         if (hdc_params_check(&pr, &pm, &full) != HDC_OK) return -1.0;
                         for (int a = 0; a < 3; ++a) full.tile[a] = pm.tile[a];
                         return cost(&pr, &full, ctx);
                     },
                     best, best_ms);
}

hdc_status hdc_predictor_load(hdc_predictor_t* out, const char* path) {
    if (!out || !path) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    FILE* fh = fopen(path, "rb");
    if (!fh) return fail(HDC_ERR_INVALID_ARG, "cannot open %s", path);
    char magic[8];
    int32_t ver = 0, n = 0;
    bool ok = fread(magic, 1, 8, fh) == 8 && !memcmp(magic, "HDCMLP01", 8) && fread(&ver, 4, 1, fh) == 1 &&
              fread(&n, 4, 1, fh) == 1 && (ver == 1 || ver == 2) && n >= 1 && n <= 16;
    std::vector<int32_t> sz(ok ? n + 1 : 0);
    if (ok) ok = fread(sz.data(), 4, n + 1, fh) == (size_t)(n + 1);
    if (ok) ok = sz[0] == kFeatures && (sz[n] == kClasses || sz[n] == kMaxClasses);
    for (int i = 0; ok && i <= n; ++i) ok = sz[i] >= 1 && sz[i] <= 4096;
    std::vector<std::vector<float>> hw, hb;
    for (int i = 0; ok && i < n; ++i) {
        hw.emplace_back((size_t)sz[i + 1] * sz[i]);
        hb.emplace_back((size_t)sz[i + 1]);
        ok = fread(hw.back().data(), 4, hw.back().size(), fh) == hw.back().size() &&
             fread(hb.back().data(), 4, hb.back().size(), fh) == hb.back().size();
    }
    float lo[kFeatures], hi[kFeatures];
    if (ok && ver == 2)
        ok = fread(lo, 4, kFeatures, fh) == (size_t)kFeatures && fread(hi, 4, kFeatures, fh) == (size_t)kFeatures;
    fclose(fh);
    if (!ok) return fail(HDC_ERR_INVALID_ARG, "%s is not a predictor checkpoint (format 1 or 2)", path);
    hdc_predictor_s* P = new hdc_predictor_s();
    P->sizes.assign(sz.begin(), sz.end());
    P->ranged = ver == 2;
    if (P->ranged) {
        std::memcpy(P->lo, lo, sizeof lo);
        std::memcpy(P->hi, hi, sizeof hi);
    }
    int wmax = 0;
    for (int v : sz) wmax = std::max(wmax, v);
    auto up = [&](const std::vector<float>& h, float** d) -> hipError_t {
        hipError_t e = hipMalloc(d, h.size() * 4);
        if (e == hipSuccess) e = hipMemcpy(*d, h.data(), h.size() * 4, hipMemcpyHostToDevice);
        return e;
    };
    hipError_t e = hipStreamCreate(&P->s);
    for (int i = 0; e == hipSuccess && i < n; ++i) {
        float *w = nullptr, *bb = nullptr;
        e = up(hw[i], &w);
        P->W.push_back(w);
        if (e == hipSuccess) e = up(hb[i], &bb);
        P->b.push_back(bb);
    }
    if (e == hipSuccess) e = hipMalloc(&P->x, (size_t)3 * kFeatures * 4);
    if (e == hipSuccess) e = hipMalloc(&P->y0, (size_t)3 * wmax * 4);
    if (e == hipSuccess) e = hipMalloc(&P->y1, (size_t)3 * wmax * 4);
    if (e == hipSuccess) e = hipMalloc(&P->P, (size_t)3 * kMaxClasses * 4);
    if (e != hipSuccess) {
        delete P;
        return fail(HDC_ERR_HIP, "predictor upload: %s", hipGetErrorString(e));
    }
    *out = P;
    return HDC_OK;
}

hdc_status hdc_predict(hdc_predictor_t P, const hdc_problem* prob, hdc_params* out, float* confidence) {
    if (!P || !prob || !out) return fail(HDC_ERR_INVALID_ARG, "NULL argument");
    const int nd = prob->ndim;
    if (nd < 1 || nd > 3) return fail(HDC_ERR_INVALID_ARG, "ndim = %d must be 1..3", nd);
    for (int a = 0; a < nd; ++a)
        if (prob->L[a] < 1 || prob->M[a] < 1) return fail(HDC_ERR_INVALID_ARG, "extents must be >= 1");
    float X[3 * kFeatures];
    for (int a = 0; a < nd; ++a) features(*prob, a, X + a * kFeatures);
    HIP_TRY(hipMemcpyAsync(P->x, X, (size_t)nd * kFeatures * 4, hipMemcpyHostToDevice, P->s));
    const int n = (int)P->W.size();
    const float* in = P->x;
    float* bufs[2] = {P->y0, P->y1};
    for (int i = 0; i < n; ++i) {
        float* o = bufs[i & 1];
        hdc_status st = hdc_mlp_linear_forward(in, P->W[i], P->b[i], o, nd, P->sizes[i], P->sizes[i + 1],
                                               i < n - 1 ? 1 : 0, P->s);
        if (st != HDC_OK) return st;
        in = o;
    }
    const int nc = P->sizes.back();  // kClasses, or kMaxClasses with the explicit class
    hdc_status st = hdc_mlp_softmax_xent(in, nullptr, P->P, nullptr, nullptr, nd, nc, P->s);
    if (st != HDC_OK) return st;
    float prob_h[3 * kMaxClasses];
    HIP_TRY(hipMemcpyAsync(prob_h, P->P, (size_t)nd * nc * 4, hipMemcpyDeviceToHost, P->s));
    HIP_TRY(hipStreamSynchronize(P->s));
    Cand c;
    for (int a = 0; a < nd; ++a) {
        int ci = 0;
        for (int k = 1; k < nc; ++k)
            if (prob_h[a * nc + k] > prob_h[a * nc + ci]) ci = k;
        if (ci == kClasses) {
            // explicit padding: one residue covering max(M, 2L - 1)
            c.m[a] = pow2_ceil(std::max(prob->M[a], 2 * prob->L[a] - 1));
            while (c.m[a] > axis_limit(*prob, a)) c.m[a] /= 2;
            while (cdiv(prob->M[a], c.m[a]) < cdiv(prob->L[a], c.m[a])) c.m[a] *= 2;
            c.D[a] = 1;
        } else {
            c.m[a] = m_for_class(*prob, a, kPClasses[ci / 2]);
            const int64_t q = cdiv(prob->M[a], c.m[a]);
            c.D[a] = (ci % 2 == 0) ? q : 1;
        }
        // an axis whose features leave the training range abstains (confidence 0)
        bool inside = true;
        for (int k = 0; P->ranged && k < kFeatures; ++k) {
            const float x = X[a * kFeatures + k];
            inside = inside && x >= P->lo[k] - kRangeMargin && x <= P->hi[k] + kRangeMargin;
        }
        if (confidence) confidence[a] = inside ? prob_h[a * nc + ci] : 0.f;
    }
    hdc_params in_p = to_params(c), full{};
    st = hdc_params_check(prob, &in_p, &full);
    if (st != HDC_OK) return st;
    for (int a = 0; a < 3; ++a) full.tile[a] = 0;
    *out = full;
    return HDC_OK;
}

hdc_status hdc_predictor_destroy(hdc_predictor_t P) {
    delete P;
    return HDC_OK;
}

hdc_status hdc_batch_db_choose(int64_t n, const int64_t* L, const int64_t* M, hdc_dtype dtype, const char* db,
                               const char* device, const char* build, int64_t* m) {
    if (n < 1 || !L || !m) return fail(HDC_ERR_INVALID_ARG, "bad batch arguments");
    if (dtype != HDC_C64 && dtype != HDC_C128) return fail(HDC_ERR_INVALID_ARG, "bad dtype");
    std::map<int64_t, std::pair<double, int64_t>> best;
    if (db) best = bucket_best(db, dtype, device ? std::string(device) : device_name(),
                               build ? std::string(build) : std::string(hdc_build_id()));
    for (int64_t i = 0; i < n; ++i) {
        if (L[i] < 1) return fail(HDC_ERR_INVALID_ARG, "problem %lld: L = %lld", (long long)i, (long long)L[i]);
        const bool full = !M || M[i] == 2 * L[i] - 1;
        auto it = best.find(pow2_ceil(L[i]));
        hdc_axis_desc d{};
        // a recorded m that this problem cannot take (a row written for other
        // lengths or by hand) leaves the problem at the default
        if (full && it != best.end() &&
            hdc_derive(L[i], 2 * L[i] - 1, it->second.second, 0, 0, 1, 0, dtype, &d) == HDC_OK) {
            m[i] = it->second.second;
        } else {
            hdc_status st = hdc_batch_default_m(L[i], &m[i]);
            if (st != HDC_OK) return st;
        }
    }
    return HDC_OK;
}

hdc_status hdc_batch_db_record(const char* db, int64_t bucket, hdc_dtype dtype, int64_t m, double ms,
                               const char* device, const char* build) {
    if (!db) return fail(HDC_ERR_INVALID_ARG, "NULL database path");
    if (bucket < 1 || (bucket & (bucket - 1)) != 0)
        return fail(HDC_ERR_INVALID_ARG, "bucket = %lld must be a power of two", (long long)bucket);
    if (m < 1 || !(ms >= 0)) return fail(HDC_ERR_INVALID_ARG, "m = %lld, ms = %g", (long long)m, ms);
    if (dtype != HDC_C64 && dtype != HDC_C128) return fail(HDC_ERR_INVALID_ARG, "bad dtype");
    const std::string dev = device ? std::string(device) : device_name();
    const std::string bld = build ? std::string(build) : std::string(hdc_build_id());
    FILE* fh = fopen(db, "a+");
    if (!fh) return fail(HDC_ERR_INVALID_ARG, "cannot open %s", db);
    // a record cut short by a kill leaves no newline: start a fresh line
    if (fseek(fh, -1, SEEK_END) == 0) {
        const int last = fgetc(fh);
        if (last != '\n' && last != EOF) fputc('\n', fh);
    }
    fseek(fh, 0, SEEK_END);
    fprintf(fh, "{\"key\": %s, \"params\": {\"m\": %lld}, \"ms\": %.9g, \"device\": %s, \"build\": %s, \"t\": %lld}\n",
            jstr(bucket_key(bucket, dtype)).c_str(), (long long)m, ms, jstr(dev).c_str(), jstr(bld).c_str(),
            (long long)time(nullptr));
    fclose(fh);
    return HDC_OK;
}

hdc_status hdc_batch_plan_db(hdc_batch_t* out, int64_t n, const int64_t* L, const int64_t* M, hdc_dtype dtype,
                             const char* db) {
    if (!out) return fail(HDC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || !L) return fail(HDC_ERR_INVALID_ARG, "bad batch arguments");
    std::vector<int64_t> m((size_t)n);
    hdc_status st = hdc_batch_db_choose(n, L, M, dtype, db, nullptr, nullptr, m.data());
    if (st != HDC_OK) return st;
    return hdc_batch_plan(out, n, L, M, m.data(), dtype);
}

}  // extern "C"
