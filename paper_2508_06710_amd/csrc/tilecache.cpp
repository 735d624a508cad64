// Tile cache files: the autotuners' choices (SpMM tile, CG tile) stored in a
// JSON object keyed by device architecture, precision and operator shape, so
// that an operator of a known shape takes its tile without timing anything.
// The file is shared with the Python side (the same keys and layout): every
// entry is an object holding at least "tile" (the 7 integers of fvx_tile in
// field order); other members ("us", "us_per_iter", "candidates", "source")
// are kept as they are when the file is rewritten.  Files are written with
// sorted keys and one-space indentation, then moved over the old file.
#include <algorithm>
#include <cctype>
#include <charconv>
#include <cstdio>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace fvx {
namespace {

// A JSON value.  Numbers keep their text, so values read from a file are
// written back unchanged.
struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    std::string text;  // Bool: "true"/"false"; Num: the number's text; Str: the decoded string
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;

    JVal *member(const std::string &k) {
        for (auto &m : obj)
            if (m.first == k) return &m.second;
        return nullptr;
    }
    void set(const std::string &k, JVal v) {
        if (JVal *p = member(k))
            *p = std::move(v);
        else
            obj.emplace_back(k, std::move(v));
    }
};

JVal num(double v) {
    char b[32];
    const auto r = std::to_chars(b, b + sizeof b, v);  // shortest text that reads back to v
    JVal j;
    j.kind = JVal::Num;
    j.text.assign(b, r.ptr);
    if (j.text.find_first_of(".eEn") == std::string::npos) j.text += ".0";  // a float stays a float
    return j;
}

JVal num(int64_t v) {
    JVal j;
    j.kind = JVal::Num;
    j.text = std::to_string(v);
    return j;
}

struct Parser {
    const std::string &s;
    size_t i = 0;

    [[noreturn]] void fail(const char *what) const {
        throw Error(FVX_E_IO, std::string("tile cache: ") + what + " at offset " + std::to_string(i));
    }
    void ws() {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
    }
    bool eat(char c) {
        ws();
        if (i < s.size() && s[i] == c) {
            ++i;
            return true;
        }
        return false;
    }
    std::string str() {
        if (!eat('"')) fail("expected a string");
        std::string out;
        while (i < s.size() && s[i] != '"') {
            char c = s[i++];
            if (c == '\\') {
                if (i >= s.size()) fail("bad escape");
                const char e = s[i++];
                switch (e) {
                    case '"': case '\\': case '/': out += e; break;
                    case 'b': out += '\b'; break;
                    case 'f': out += '\f'; break;
                    case 'n': out += '\n'; break;
                    case 'r': out += '\r'; break;
                    case 't': out += '\t'; break;
                    case 'u': {
                        if (i + 4 > s.size()) fail("bad \\u escape");
                        unsigned cp = 0;
                        const auto r = std::from_chars(s.data() + i, s.data() + i + 4, cp, 16);
                        if (r.ec != std::errc() || r.ptr != s.data() + i + 4) fail("bad \\u escape");
                        i += 4;
                        if (cp >= 0x80) fail("non-ASCII \\u escape");
                        out += char(cp);
                        break;
                    }
                    default: fail("bad escape");
                }
            } else {
                out += c;
            }
        }
        if (i >= s.size()) fail("unterminated string");
        ++i;
        return out;
    }
    JVal value() {
        ws();
        if (i >= s.size()) fail("unexpected end");
        JVal v;
        const char c = s[i];
        if (c == '{') {
            ++i;
            v.kind = JVal::Obj;
            if (eat('}')) return v;
            do {
                std::string k = str();
                if (!eat(':')) fail("expected ':'");
                v.obj.emplace_back(std::move(k), value());
            } while (eat(','));
            if (!eat('}')) fail("expected '}'");
        } else if (c == '[') {
            ++i;
            v.kind = JVal::Arr;
            if (eat(']')) return v;
            do v.arr.push_back(value());
            while (eat(','));
            if (!eat(']')) fail("expected ']'");
        } else if (c == '"') {
            v.kind = JVal::Str;
            v.text = str();
        } else if (s.compare(i, 4, "true") == 0 || s.compare(i, 5, "false") == 0) {
            v.kind = JVal::Bool;
            v.text = s[i] == 't' ? "true" : "false";
            i += v.text.size();
        } else if (s.compare(i, 4, "null") == 0) {
            i += 4;
        } else {
            const size_t b = i;
            while (i < s.size() && (std::isdigit(static_cast<unsigned char>(s[i])) || s[i] == '-' || s[i] == '+' ||
                                    s[i] == '.' || s[i] == 'e' || s[i] == 'E'))
                ++i;
            if (i == b) fail("unexpected character");
            v.kind = JVal::Num;
            v.text = s.substr(b, i - b);
        }
        return v;
    }
};

void put_str(std::ostream &o, const std::string &t) {
    o << '"';
    for (char c : t) {
        switch (c) {
            case '"': o << "\\\""; break;
            case '\\': o << "\\\\"; break;
            case '\n': o << "\\n"; break;
            case '\t': o << "\\t"; break;
            case '\r': o << "\\r"; break;
            default: o << c;
        }
    }
    o << '"';
}

// The layout of Python's json.dump(..., indent=1, sort_keys=True).
void put(std::ostream &o, const JVal &v, int level) {
    const std::string in(size_t(level + 1), ' '), out(size_t(level), ' ');
    switch (v.kind) {
        case JVal::Null: o << "null"; break;
        case JVal::Bool:
        case JVal::Num: o << v.text; break;
        case JVal::Str: put_str(o, v.text); break;
        case JVal::Arr:
            if (v.arr.empty()) {
                o << "[]";
                break;
            }
            o << "[\n";
            for (size_t k = 0; k < v.arr.size(); ++k) {
                o << in;
                put(o, v.arr[k], level + 1);
                o << (k + 1 < v.arr.size() ? ",\n" : "\n");
            }
            o << out << ']';
            break;
        case JVal::Obj: {
            if (v.obj.empty()) {
                o << "{}";
                break;
            }
            std::vector<const std::pair<std::string, JVal> *> m;
            for (const auto &e : v.obj) m.push_back(&e);
            std::sort(m.begin(), m.end(), [](auto *a, auto *b) { return a->first < b->first; });
            o << "{\n";
            for (size_t k = 0; k < m.size(); ++k) {
                o << in;
                put_str(o, m[k]->first);
                o << ": ";
                put(o, m[k]->second, level + 1);
                o << (k + 1 < m.size() ? ",\n" : "\n");
            }
            o << out << '}';
            break;
        }
    }
}

JVal read_cache(const char *path) {
    JVal doc;
    doc.kind = JVal::Obj;
    std::ifstream f(path, std::ios::binary);
    if (!f) return doc;  // no file yet: an empty cache
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string text = ss.str();
    Parser p{text};
    doc = p.value();
    p.ws();
    if (doc.kind != JVal::Obj || p.i != text.size()) throw Error(FVX_E_IO, std::string(path) + " is not a JSON object");
    return doc;
}

void write_cache(const char *path, const JVal &doc) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
        FVX_REQUIRE(f, FVX_E_IO, "cannot write " + tmp);
        put(f, doc, 0);
        f.flush();
        FVX_REQUIRE(f.good(), FVX_E_IO, "writing " + tmp + " failed");
    }
    FVX_REQUIRE(std::rename(tmp.c_str(), path) == 0, FVX_E_IO, "cannot replace " + std::string(path));
}

// The device's architecture name without its feature suffix ("gfx950").
std::string arch_name() {
    int dev = 0;
    FVX_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FVX_HIP(hipGetDeviceProperties(&prop, dev));
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

std::string tile_key(const fvx_op *op, int dtype, bool cg) {
    std::string k = cg ? "cg|" : "";
    k += arch_name() + "|" + (dtype == FVX_F64 ? "f64" : "f32") + "|k=" + std::to_string(op->k) +
         "|ld=" + std::to_string(op->ld) + "|n_b=" + std::to_string(op->n_b) + "|nnz_b=" + std::to_string(op->nnz_b);
    k += cg ? "|coupling=" + std::to_string(op->coupling) : "|stencil=" + std::to_string(op->stencil);
    return k;
}

// The cached tile of `key` (false when absent or not 6-7 integers).
bool cached_tile(JVal &doc, const std::string &key, fvx_tile &t) {
    JVal *e = doc.member(key);
    if (!e || e->kind != JVal::Obj) return false;
    JVal *a = e->member("tile");
    if (!a || a->kind != JVal::Arr || a->arr.size() < 6 || a->arr.size() > 7) return false;
    int v[7] = {0, 0, 0, 0, 0, 0, 0};
    for (size_t i = 0; i < a->arr.size(); ++i) {
        if (a->arr[i].kind != JVal::Num) return false;
        const std::string &x = a->arr[i].text;
        const auto r = std::from_chars(x.data(), x.data() + x.size(), v[i]);
        if (r.ec != std::errc() || r.ptr != x.data() + x.size()) return false;  // not an integer: tuned again
    }
    t = fvx_tile{v[0], v[1], v[2], v[3], v[4], v[5], v[6]};
    return true;
}

JVal tile_json(const fvx_tile &t) {
    JVal a;
    a.kind = JVal::Arr;
    for (int x : {t.vec, t.lanes_per_row, t.block, t.xcd_remap, t.max_blocks, t.stage_lds, t.nt_store})
        a.arr.push_back(num(int64_t(x)));
    return a;
}

std::mutex g_cache_mu;  // one writer at a time within the process

template <class Tune>
int cached(fvx_op *op, int dtype, const char *path, bool cg, fvx_tile *tile, int *from_cache, Tune tune_fn) {
    FVX_REQUIRE(op, FVX_E_ARG, "op is NULL");
    FVX_REQUIRE(dtype == FVX_F64 || (dtype == FVX_F32 && op->has_f32), FVX_E_ARG, "bad dtype for this op");
    const std::string key = tile_key(op, dtype, cg);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    JVal doc;
    doc.kind = JVal::Obj;
    if (path) doc = read_cache(path);
    fvx_tile t{};
    if (cached_tile(doc, key, t)) {
        if (cg) t.nt_store = 0;
        const int rc = cg ? fvx_op_set_cg_tile(op, dtype, &t) : fvx_op_set_tile(op, dtype, &t);
        if (rc == FVX_OK) {
            if (tile) *tile = t;
            if (from_cache) *from_cache = 1;
            return FVX_OK;
        }
        // a stored tile this build rejects is tuned again and replaced
    }
    std::vector<fvx_tune_result> res(1024);
    int n = 0;
    const int rc = tune_fn(res.data(), int(res.size()), &n);
    if (rc != FVX_OK) return rc;
    FVX_REQUIRE(n >= 1, FVX_E_UNSUPPORTED, "the autotuner tried no candidate");
    double best = res[0].us;
    for (int i = 1; i < std::min(n, int(res.size())); ++i) best = std::min(best, res[i].us);
    FVX_REQUIRE((cg ? fvx_op_get_cg_tile(op, dtype, &t) : fvx_op_get_tile(op, dtype, &t)) == FVX_OK, FVX_E_ARG,
                "reading the tuned tile failed");
    if (path) {
        JVal e;
        e.kind = JVal::Obj;
        if (JVal *old = doc.member(key))
            if (old->kind == JVal::Obj) e = *old;
        e.set("tile", tile_json(t));
        e.set(cg ? "us_per_iter" : "us", num(best));
        e.set("candidates", num(int64_t(n)));
        doc.set(key, std::move(e));
        write_cache(path, doc);
    }
    if (tile) *tile = t;
    if (from_cache) *from_cache = 0;
    return FVX_OK;
}

}  // namespace
}  // namespace fvx

extern "C" int fvx_tune_cached(fvx_op *op, int dtype, const char *cache_path, void *scratch, size_t scratch_bytes,
                               int reps, void *stream, fvx_tile *tile, int *from_cache) {
    return fvx::guard([&] {
        return fvx::cached(op, dtype, cache_path, false, tile, from_cache, [&](fvx_tune_result *r, int m, int *n) {
            return fvx_tune(op, dtype, scratch, scratch_bytes, reps, stream, r, m, n);
        });
    });
}

extern "C" int fvx_tune_cg_cached(fvx_op *op, int dtype, const char *cache_path, void *ws, size_t ws_bytes, int iters,
                                  void *stream, fvx_tile *tile, int *from_cache) {
    return fvx::guard([&] {
        return fvx::cached(op, dtype, cache_path, true, tile, from_cache, [&](fvx_tune_result *r, int m, int *n) {
            return fvx_tune_cg(op, dtype, ws, ws_bytes, iters, stream, r, m, n);
        });
    });
}
