// On-disk cache of the FP64 operator precomputation.
//
// The translation operators of Sec. II (check-to-equivalent pseudo-inverses,
// M2M/L2L, the V-list translations and their compressed basis, the periodic
// far images) depend only on the order p, the boundary and two cut
// tolerances, yet take seconds to build in FP64 (about 1.5 s at p = 8,
// 5.5 s at p = 10).  A process that finds a matching file loads it instead.
//
// File: one per operator set, named by its parameters (exact bit patterns of
// the tolerances) and by a hash of the sources that compute the operators,
// so a library built from changed operator code never reads an older file.
// Content (native byte order): 8-byte magic, 64-byte source-hash field, the
// parameters, the array sizes and arrays (each a uint64 element count and
// the elements), then a 64-bit hash of everything before it.  A file whose
// magic, parameters, sizes or hash do not match is ignored and rewritten.
// Writers write a private temporary file and rename it into place, so
// concurrent processes see either no file or a whole one.  The cache is best
// effort: a directory that cannot be created or written only costs the
// rebuild.
#include <cerrno>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>
#include <atomic>

#include "internal.hpp"

#ifndef KAFMM_OPS_SOURCE_HASH
#define KAFMM_OPS_SOURCE_HASH "unversioned"
#endif

namespace kafmm {
namespace {

constexpr char kMagicOps[8] = {'K', 'A', 'F', 'M', 'M', 'O', 'P', 'S'};
constexpr char kMagicStk[8] = {'K', 'A', 'F', 'M', 'M', 'S', 'T', 'K'};

// Streaming 64-bit hash over 8-byte words (multiply-xorshift mixing): the
// value depends only on the byte sequence, not on how it was split into
// add() calls; finish() mixes in the tail and the length.
struct Hash64 {
    uint64_t h = 0x9e3779b97f4a7c15ull, pend = 0, total = 0;
    void mix(uint64_t w) {
        h ^= w + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        h *= 0xff51afd7ed558ccdull;
        h ^= h >> 33;
    }
    void byte(unsigned char c) {
        pend |= uint64_t(c) << (8 * (total & 7));
        if ((++total & 7) == 0) {
            mix(pend);
            pend = 0;
        }
    }
    void add(const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        size_t i = 0;
        for (; i < n && (total & 7) != 0; ++i) byte(b[i]);
        for (; i + 8 <= n; i += 8) {          // whole words (little-endian byte order, as byte() builds them)
            uint64_t w;
            std::memcpy(&w, b + i, 8);
            mix(w);
            total += 8;
        }
        for (; i < n; ++i) byte(b[i]);
    }
    uint64_t finish() const {
        Hash64 t = *this;
        t.mix(t.pend ^ (t.total << 3));
        return t.h;
    }
};

uint64_t bits(double v) {
    uint64_t u;
    std::memcpy(&u, &v, 8);
    return u;
}

// Serialiser that feeds every byte to the hash and, when a file is given, to it.
struct Sink {
    FILE *f = nullptr;
    Hash64 hash;
    bool ok = true;
    void put(const void *p, size_t n) {
        hash.add(p, n);
        if (f && n && std::fwrite(p, 1, n, f) != n) ok = false;
    }
    template <class T> void scalar(T v) { put(&v, sizeof(T)); }
    template <class T> void array(const std::vector<T> &a) {
        scalar<uint64_t>(a.size());
        put(a.data(), a.size() * sizeof(T));
    }
};

// Reader over a whole file in memory; every read is bounds checked.
struct Source {
    const std::vector<unsigned char> &buf;
    size_t pos = 0;
    bool ok = true;
    explicit Source(const std::vector<unsigned char> &b) : buf(b) {}
    void get(void *p, size_t n) {
        if (!ok || n > buf.size() - pos) {
            ok = false;
            return;
        }
        std::memcpy(p, buf.data() + pos, n);
        pos += n;
    }
    template <class T> T scalar() {
        T v{};
        get(&v, sizeof(T));
        return v;
    }
    template <class T> void array(std::vector<T> &a, uint64_t expect) {
        const uint64_t n = scalar<uint64_t>();
        if (!ok || n != expect || n > (buf.size() - pos) / sizeof(T)) {
            ok = false;
            return;
        }
        a.resize(n);
        get(a.data(), n * sizeof(T));
    }
};

void header(Sink &s, const char magic[8]) {
    s.put(magic, 8);
    char src[64] = {};
    std::strncpy(src, KAFMM_OPS_SOURCE_HASH, sizeof(src) - 1);
    s.put(src, sizeof(src));
}

bool header_ok(Source &r, const char magic[8]) {
    char m[8], src[64], want[64] = {};
    r.get(m, 8);
    r.get(src, 64);
    std::strncpy(want, KAFMM_OPS_SOURCE_HASH, sizeof(want) - 1);
    return r.ok && std::memcmp(m, magic, 8) == 0 && std::memcmp(src, want, 64) == 0;
}

void write_ops(Sink &s, const Operators &o, bool periodic) {
    header(s, kMagicOps);
    s.scalar<int32_t>(o.p);
    s.scalar<int32_t>(periodic ? 1 : 0);
    s.scalar<uint64_t>(bits(o.svd_tol));
    s.scalar<uint64_t>(bits(o.m2l_tol));
    s.scalar<int32_t>(o.M);
    s.scalar<int32_t>(o.Mp);
    s.scalar<int32_t>(o.rank);
    s.scalar<int32_t>(o.kc);
    s.array(o.grid);
    s.array(o.up1);
    s.array(o.up2);
    s.array(o.m2m);
    s.array(o.l2l_cc);
    s.array(o.m2l);
    s.array(o.cbasis);
    s.array(o.m2l_c);
    s.array(o.t_m2l);
}

void write_stk(Sink &s, int p, double svd_tol, bool doubly, const std::vector<double> &Q,
               const std::vector<double> &X, const std::vector<double> &Z) {
    header(s, kMagicStk);
    s.scalar<int32_t>(p);
    s.scalar<int32_t>(doubly ? 1 : 0);
    s.scalar<uint64_t>(bits(svd_tol));
    s.scalar<int32_t>(int32_t(X.size() / 3));
    s.array(Q);
    s.array(X);
    s.array(Z);
}

bool read_file(const std::string &path, std::vector<unsigned char> &buf) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return false;
    bool ok = std::fseek(f, 0, SEEK_END) == 0;
    const long n = ok ? std::ftell(f) : -1;
    ok = ok && n > 16 && std::fseek(f, 0, SEEK_SET) == 0;
    if (ok) {
        buf.resize(size_t(n));
        ok = std::fread(buf.data(), 1, buf.size(), f) == buf.size();
    }
    std::fclose(f);
    return ok;
}

// The trailing 8 bytes hold the hash of everything before them.
bool trailer_ok(const std::vector<unsigned char> &buf, size_t body) {
    if (body + 8 != buf.size()) return false;
    Hash64 h;
    h.add(buf.data(), body);
    uint64_t stored;
    std::memcpy(&stored, buf.data() + body, 8);
    return stored == h.finish();
}

void make_dirs(const std::string &dir) {
    for (size_t i = 1; i <= dir.size(); ++i)
        if (i == dir.size() || dir[i] == '/') ::mkdir(dir.substr(0, i).c_str(), 0755);
}

// Writes through a private temporary file renamed into place.
template <class F> void store(const std::string &dir, const std::string &name, F &&write) {
    static std::atomic<unsigned> counter{0};
    make_dirs(dir);
    const std::string path = dir + "/" + name;
    const std::string tmp = path + ".tmp." + std::to_string(::getpid()) + "." + std::to_string(counter++);
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    Sink s;
    s.f = f;
    write(s);
    const uint64_t h = s.hash.finish();
    bool ok = s.ok && std::fwrite(&h, 1, 8, f) == 8;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

std::string hex64(uint64_t v) {
    char b[17];
    std::snprintf(b, sizeof(b), "%016llx", static_cast<unsigned long long>(v));
    return b;
}

std::string source_tag() {
    std::string t = KAFMM_OPS_SOURCE_HASH;
    return t.substr(0, 16);
}

}  // namespace

std::string default_operator_cache_dir() {
    if (const char *e = std::getenv("STKFMM_OPERATOR_CACHE")) return e;   // "" disables the cache
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/stkfmm_operators";
    if (const char *h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/stkfmm_operators";
    return "";
}

uint64_t operators_digest(const Operators &ops, bool periodic) {
    Sink s;
    write_ops(s, ops, periodic);
    return s.hash.finish();
}

uint64_t stokes_far_digest(int p, double svd_tol, bool doubly, const std::vector<double> &Q,
                           const std::vector<double> &X, const std::vector<double> &Z) {
    Sink s;
    write_stk(s, p, svd_tol, doubly, Q, X, Z);
    return s.hash.finish();
}

std::string cached_operators(const std::string &dir, int p, double svd_tol, bool periodic, double m2l_tol,
                             Operators &ops, bool *loaded) {
    if (loaded) *loaded = false;
    const std::string name = "ops_p" + std::to_string(p) + (periodic ? "_pxyz_" : "_open_") + hex64(bits(svd_tol)) +
                             "_" + hex64(bits(m2l_tol)) + "_" + source_tag() + ".bin";
    std::vector<unsigned char> buf;
    if (!dir.empty() && read_file(dir + "/" + name, buf) && trailer_ok(buf, buf.size() - 8)) {
        Source r(buf);
        Operators o;
        bool ok = header_ok(r, kMagicOps);
        o.p = r.scalar<int32_t>();
        const bool per = r.scalar<int32_t>() != 0;
        const uint64_t st = r.scalar<uint64_t>(), mt = r.scalar<uint64_t>();
        o.M = r.scalar<int32_t>();
        o.Mp = r.scalar<int32_t>();
        o.rank = r.scalar<int32_t>();
        o.kc = r.scalar<int32_t>();
        ok = ok && r.ok && o.p == p && per == periodic && st == bits(svd_tol) && mt == bits(m2l_tol) &&
             o.M == 6 * (p - 1) * (p - 1) + 2 && o.Mp == (o.M + 31) / 32 * 32 && o.rank > 0 && o.rank <= o.M &&
             o.kc >= 0 && o.kc <= o.M;
        if (ok) {
            const uint64_t M = uint64_t(o.M), Mp = uint64_t(o.Mp), R = uint64_t(o.rank), K = uint64_t(o.kc);
            r.array(o.grid, 3 * M);
            r.array(o.up1, M * R);
            r.array(o.up2, R * M);
            r.array(o.m2m, 8 * Mp * Mp);
            r.array(o.l2l_cc, 8 * M * M);
            r.array(o.m2l, K == 0 ? 343 * Mp * Mp : 0);
            r.array(o.cbasis, K > 0 ? Mp * K : 0);
            r.array(o.m2l_c, K > 0 ? 343 * K * K : 0);
            r.array(o.t_m2l, periodic ? M * M : 0);
            ok = r.ok && r.pos + 8 == buf.size();
        }
        if (ok) {
            o.svd_tol = svd_tol;
            o.m2l_tol = m2l_tol;
            ops = std::move(o);
            if (loaded) *loaded = true;
            return "";
        }
    }
    std::string e = build_operators(p, svd_tol, periodic, ops, m2l_tol);
    if (e.empty() && !dir.empty()) store(dir, name, [&](Sink &s) { write_ops(s, ops, periodic); });
    return e;
}

std::string cached_periodic_stokes(const std::string &dir, int p, double svd_tol, bool doubly, std::vector<double> &Q,
                                   std::vector<double> &X, std::vector<double> &Z, bool *loaded) {
    if (loaded) *loaded = false;
    const std::string name = "stkfar_p" + std::to_string(p) + (doubly ? "_pxy_" : "_pxyz_") + hex64(bits(svd_tol)) +
                             "_" + source_tag() + ".bin";
    std::vector<unsigned char> buf;
    if (!dir.empty() && read_file(dir + "/" + name, buf) && trailer_ok(buf, buf.size() - 8)) {
        Source r(buf);
        bool ok = header_ok(r, kMagicStk);
        const int pp = r.scalar<int32_t>();
        const bool dd = r.scalar<int32_t>() != 0;
        const uint64_t st = r.scalar<uint64_t>();
        const int M = r.scalar<int32_t>();
        ok = ok && r.ok && pp == p && dd == doubly && st == bits(svd_tol) && M == 6 * (p - 1) * (p - 1) + 2;
        std::vector<double> q, x, z;
        if (ok) {
            r.array(q, 9 * uint64_t(M) * M);
            r.array(x, 3 * uint64_t(M));
            r.array(z, 3 * uint64_t(M));
            ok = r.ok && r.pos + 8 == buf.size();
        }
        if (ok) {
            Q = std::move(q);
            X = std::move(x);
            Z = std::move(z);
            if (loaded) *loaded = true;
            return "";
        }
    }
    std::string e = build_periodic_stokes(p, svd_tol, doubly, Q, X, Z);
    if (e.empty() && !dir.empty()) store(dir, name, [&](Sink &s) { write_stk(s, p, svd_tol, doubly, Q, X, Z); });
    return e;
}

}  // namespace kafmm
