// Tuning table of libltl: launch shapes keyed by method, element type, epilogue class, radius,
// grid-size bucket, boundary and batched, read from two JSON files (the user cache, then the
// table shipped beside the library), and the LTL_TILE override. Host-only code: nothing here
// touches the device, so the lookup logic is testable without a GPU.
#include <dlfcn.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "host_common.h"
#include "ltl.h"
#include "tuning_cache.h"

namespace ltl {
namespace host {

// ------------------------------------------------------------------ a small JSON reader/writer
// Enough of JSON for the table files: objects, arrays, strings without escapes other than \" and
// \\, numbers, true / false / null.
struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const std::string &k) const {
        for (auto &kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

namespace {

struct Parser {
    const std::string &s;
    size_t i = 0;
    bool ok = true;
    explicit Parser(const std::string &t) : s(t) {}
    void ws() {
        while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) { ++i; return true; }
        return false;
    }
    std::string string_lit() {
        std::string out;
        if (!eat('"')) { ok = false; return out; }
        while (i < s.size() && s[i] != '"') {
            if (s[i] == '\\' && i + 1 < s.size()) ++i;
            out.push_back(s[i++]);
        }
        if (i >= s.size()) { ok = false; return out; }
        ++i;
        return out;
    }
    JVal value(int depth = 0) {
        JVal v;
        if (depth > 16) { ok = false; return v; }
        ws();
        if (i >= s.size()) { ok = false; return v; }
        const char c = s[i];
        if (c == '{') {
            ++i;
            v.kind = JVal::OBJ;
            if (eat('}')) return v;
            do {
                std::string k = string_lit();
                if (!ok || !eat(':')) { ok = false; return v; }
                v.obj.emplace_back(k, value(depth + 1));
                if (!ok) return v;
            } while (eat(','));
            if (!eat('}')) ok = false;
        } else if (c == '[') {
            ++i;
            v.kind = JVal::ARR;
            if (eat(']')) return v;
            do {
                v.arr.push_back(value(depth + 1));
                if (!ok) return v;
            } while (eat(','));
            if (!eat(']')) ok = false;
        } else if (c == '"') {
            v.kind = JVal::STR;
            v.str = string_lit();
        } else if (s.compare(i, 4, "true") == 0) {
            v.kind = JVal::BOOL; v.b = true; i += 4;
        } else if (s.compare(i, 5, "false") == 0) {
            v.kind = JVal::BOOL; i += 5;
        } else if (s.compare(i, 4, "null") == 0) {
            i += 4;
        } else {
            const char *p = s.c_str() + i;
            char *e = nullptr;
            v.num = std::strtod(p, &e);
            if (e == p) { ok = false; return v; }
            v.kind = JVal::NUM;
            i += (size_t)(e - p);
        }
        return v;
    }
};

bool read_file(const std::string &path, std::string *out) {
    std::ifstream f(path);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    *out = ss.str();
    return true;
}

const char *method_name(int m) {
    return m == LTL_CAT_I8 ? "cat_i8" : m == LTL_CAT_F16 ? "cat_f16" : m == LTL_CAT_F8 ? "cat_f8" : "direct";
}
const char *elem_name(int method, int elem) {
    if (method == LTL_DIRECT) return "direct";
    return elem == ELEM_I8 ? "i8" : elem == ELEM_I8W ? "i8w" : elem == ELEM_I8X ? "i8x" : elem == ELEM_F16 ? "f16" : "f8";
}
const char *epi_name(int epi) {
    return epi == EPI_BYTE ? "byte" : epi == EPI_HALF ? "half" : epi_decays(epi) ? "decay" : "win";
}

struct Entry {
    TuneKey key;
    ltl_tuning_t t;
    double ms = 0;
};

bool entry_of(const JVal &e, Entry *out) {
    if (e.kind != JVal::OBJ) return false;
    auto str = [&](const char *k, std::string *v) {
        const JVal *x = e.get(k);
        if (!x || x->kind != JVal::STR) return false;
        *v = x->str;
        return true;
    };
    auto num = [&](const char *k, double *v) {
        const JVal *x = e.get(k);
        if (!x || x->kind != JVal::NUM) return false;
        *v = x->num;
        return true;
    };
    double r, bucket, batched;
    if (!str("method", &out->key.method) || !str("elem", &out->key.elem) || !str("epi", &out->key.epi) ||
        !str("boundary", &out->key.boundary) || !num("r", &r) || !num("bucket", &bucket) || !num("batched", &batched))
        return false;
    out->key.r = (int)r;
    out->key.bucket = (int)bucket;
    out->key.batched = (int)batched;
    const JVal *t = e.get("tuning");
    if (!t || t->kind != JVal::ARR || t->arr.size() < 4 || t->arr.size() > 7) return false;
    int32_t v[7] = {0, 0, 0, 0, 1, 0, 0};
    for (size_t k = 0; k < t->arr.size(); ++k) {
        if (t->arr[k].kind != JVal::NUM) return false;
        v[k] = (int32_t)t->arr[k].num;
    }
    out->t = ltl_tuning_t{v[0], v[1], v[2], v[3], v[4], v[5], v[6]};
    double ms = 0;
    if (num("ms_per_step", &ms)) out->ms = ms;
    return true;
}

std::vector<Entry> read_entries(const std::string &path) {
    std::vector<Entry> out;
    std::string text;
    if (path.empty() || !read_file(path, &text)) return out;
    Parser p(text);
    JVal root = p.value();
    if (!p.ok || root.kind != JVal::OBJ) return out;
    const JVal *es = root.get("entries");
    if (!es || es->kind != JVal::ARR) return out;
    for (auto &e : es->arr) {
        Entry x;
        if (entry_of(e, &x)) out.push_back(x);
    }
    return out;
}

std::string entry_json(const Entry &e) {
    char buf[512];
    std::snprintf(buf, sizeof(buf),
                  "{\"method\": \"%s\", \"elem\": \"%s\", \"epi\": \"%s\", \"r\": %d, \"bucket\": %d, "
                  "\"boundary\": \"%s\", \"batched\": %d, \"tuning\": [%d, %d, %d, %d, %d, %d, %d], "
                  "\"ms_per_step\": %.6g}",
                  e.key.method.c_str(), e.key.elem.c_str(), e.key.epi.c_str(), e.key.r, e.key.bucket,
                  e.key.boundary.c_str(), e.key.batched, e.t.steps_per_launch, e.t.tile_rows, e.t.tile_cols,
                  e.t.waves, e.t.use_graph, e.t.persistent, e.t.lds_pad, e.ms);
    return buf;
}

bool write_entries(const std::string &path, const std::vector<Entry> &es) {
    // create the directory chain if missing
    for (size_t k = 1; k < path.size(); ++k)
        if (path[k] == '/') (void)mkdir(path.substr(0, k).c_str(), 0755);
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\"version\": 1, \"entries\": [\n");
    for (size_t k = 0; k < es.size(); ++k)
        std::fprintf(f, "  %s%s\n", entry_json(es[k]).c_str(), k + 1 < es.size() ? "," : "");
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

bool same_class(const TuneKey &a, const TuneKey &b) {
    return a.method == b.method && a.elem == b.elem && a.epi == b.epi && a.boundary == b.boundary &&
           a.batched == b.batched;
}

}  // namespace

std::string user_cache_path() {
    const char *env = std::getenv("LTL_TUNE_CACHE");
    if (env && *env) return std::strcmp(env, "off") == 0 ? std::string() : std::string(env);
    const char *xdg = std::getenv("XDG_CACHE_HOME");
    if (xdg && *xdg) return std::string(xdg) + "/ltl/tuning.json";
    const char *home = std::getenv("HOME");
    if (home && *home) return std::string(home) + "/.cache/ltl/tuning.json";
    return std::string();
}

std::string shipped_table_path() {
    const char *env = std::getenv("LTL_TUNE_TABLE");
    if (env && *env) return env;
    Dl_info info;
    if (dladdr((const void *)&shipped_table_path, &info) && info.dli_fname) {
        std::string lib = info.dli_fname;
        const size_t slash = lib.rfind('/');
        return (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning.json";
    }
    return std::string();
}

int size_bucket(double cells) {
    if (cells < 1) cells = 1;
    return (int)std::lround(0.5 * std::log2(cells));
}

TuneKey make_key(int H, int W, const ltl_rule_t &rule, int method, int boundary, int batched) {
    TuneKey k;
    const int elem = elem_of(method, rule.R, rule.N);
    k.method = method_name(method);
    k.elem = elem_name(method, elem);
    k.epi = batched ? "mixed" : epi_name(epi_of(rule, elem));
    k.r = batched ? 0 : rule.R;
    k.bucket = size_bucket((double)H * (double)W);
    k.boundary = boundary == LTL_BOUNDARY_PERIODIC ? "periodic" : "dead";
    k.batched = batched ? 1 : 0;
    return k;
}

std::vector<ltl_tuning_t> tuning_candidates(const TuneKey &key, bool *exact) {
    struct Cand {
        int src, dr, db, order;
        ltl_tuning_t t;
    };
    std::vector<Cand> cs;
    const std::string paths[2] = {user_cache_path(), shipped_table_path()};
    int order = 0;
    for (int src = 0; src < 2; ++src)
        for (const Entry &e : read_entries(paths[src]))
            if (same_class(e.key, key))
                cs.push_back({src, std::abs(e.key.r - key.r), std::abs(e.key.bucket - key.bucket), order++, e.t});
    // nearest radius first, then nearest size bucket; the user cache wins ties
    std::stable_sort(cs.begin(), cs.end(), [](const Cand &a, const Cand &b) {
        if (a.dr != b.dr) return a.dr < b.dr;
        if (a.db != b.db) return a.db < b.db;
        return a.src < b.src;
    });
    if (exact) *exact = !cs.empty() && cs[0].dr == 0 && cs[0].db == 0;
    std::vector<ltl_tuning_t> out;
    for (auto &c : cs) out.push_back(c.t);
    return out;
}

bool store_tuning(const TuneKey &key, const ltl_tuning_t &t, double ms, std::string *err) {
    const std::string path = user_cache_path();
    if (path.empty()) {
        *err = "the user tuning cache is off (LTL_TUNE_CACHE=off) or has no path";
        return false;
    }
    std::vector<Entry> es = read_entries(path);
    Entry n;
    n.key = key;
    n.t = t;
    n.ms = ms;
    bool replaced = false;
    for (auto &e : es)
        if (same_class(e.key, key) && e.key.r == key.r && e.key.bucket == key.bucket) {
            e = n;
            replaced = true;
        }
    if (!replaced) es.push_back(n);
    if (!write_entries(path, es)) {
        *err = "cannot write the tuning cache " + path;
        return false;
    }
    return true;
}

int env_tile(ltl_tuning_t *t, std::string *err) {
    const char *env = std::getenv("LTL_TILE");
    if (!env || !*env) return 0;
    int32_t v[6] = {0, 0, 0, 0, 0, 0};
    int n = 0;
    const char *p = env;
    while (*p && n < 6) {
        char *e = nullptr;
        const long x = std::strtol(p, &e, 10);
        if (e == p || x < 0 || x > 4096) break;
        v[n++] = (int32_t)x;
        p = e;
        if (*p == ',') ++p;
        else break;
    }
    if (*p || n < 4) {
        *err = std::string("LTL_TILE must be \"T,rows,cols,waves[,persistent[,lds_pad]]\", got \"") + env + "\"";
        return -1;
    }
    *t = ltl_tuning_t{v[0], v[1], v[2], v[3], 1, v[4], v[5]};
    return 1;
}

}  // namespace host
}  // namespace ltl

using namespace ltl::host;

extern "C" {

int32_t ltl_tuning_lookup(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                          int32_t batched, ltl_tuning_t *out, int32_t *exact) {
    if (!rule || !out) return fail(LTL_ERR_ARG, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    if (exact) *exact = 0;
    if (H < 1 || W < 1) return fail(LTL_ERR_ARG, "H and W must be >= 1");
    int32_t rc = validate_rule(rule, method);
    if (rc != LTL_OK) return rc;
    bool ex = false;
    std::vector<ltl_tuning_t> c = tuning_candidates(make_key(H, W, *rule, method, boundary, batched), &ex);
    if (c.empty()) return fail(LTL_ERR_ARG, "no tuning table entry for this class");
    *out = c[0];
    if (exact) *exact = ex ? 1 : 0;
    return LTL_OK;
}

int32_t ltl_tuning_store(int32_t H, int32_t W, const ltl_rule_t *rule, int32_t method, int32_t boundary,
                         int32_t batched, const ltl_tuning_t *tuning, double ms_per_step) {
    if (!rule || !tuning) return fail(LTL_ERR_ARG, "NULL argument");
    if (H < 1 || W < 1) return fail(LTL_ERR_ARG, "H and W must be >= 1");
    int32_t rc = validate_rule(rule, method);
    if (rc != LTL_OK) return rc;
    std::string err;
    if (!store_tuning(make_key(H, W, *rule, method, boundary, batched), *tuning, ms_per_step, &err))
        return fail(LTL_ERR_ARG, err);
    return LTL_OK;
}

}  // extern "C"
