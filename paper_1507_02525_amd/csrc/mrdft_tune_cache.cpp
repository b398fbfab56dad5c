// Persistent cache of tuned forward schedules (include/mrdft_tune.h).
// Host code only: a small reader for the one JSON shape this file writes, and
// an atomic whole-file replace on store.  Anything the reader does not accept
// makes the file count as empty.
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <unistd.h>

#include "../../include/mrdft_tune.h"

namespace {

struct Entry {
    long tile_log = -1, grid = -1, order = -1, serial = -1;
    bool valid() const { return tile_log >= 0 && grid >= 0 && order >= 0 && serial >= 0; }
};

using Table = std::map<std::string, Entry>;

bool key_ok(const char* k) {
    if (!k || !*k) return false;
    for (const unsigned char* c = (const unsigned char*)k; *c; ++c)
        if (*c < 0x20 || *c == '"' || *c == '\\' || *c == 0x7f) return false;
    return true;
}

// Recursive-descent reader of exactly the accepted shape.
struct Reader {
    const std::string& s;
    size_t i = 0;
    explicit Reader(const std::string& t) : s(t) {}
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
    // strings without escapes (keys are written without '"' and '\\')
    bool str(std::string* out) {
        ws();
        if (i >= s.size() || s[i] != '"') return false;
        const size_t b = ++i;
        while (i < s.size() && s[i] != '"') {
            const unsigned char c = (unsigned char)s[i];
            if (c < 0x20 || c == '\\') return false;
            ++i;
        }
        if (i >= s.size()) return false;
        *out = s.substr(b, i - b);
        ++i;
        return true;
    }
    bool integer(long* out) {
        ws();
        const size_t b = i;
        if (i < s.size() && s[i] == '-') ++i;
        const size_t d = i;
        while (i < s.size() && s[i] >= '0' && s[i] <= '9') ++i;
        if (i == d || i - d > 9) return false;
        *out = std::strtol(s.substr(b, i - b).c_str(), nullptr, 10);
        return true;
    }
    bool entry(Entry* e) {
        if (!eat('{')) return false;
        if (eat('}')) return false;
        do {
            std::string k;
            long v = 0;
            if (!str(&k) || !eat(':') || !integer(&v)) return false;
            if (k == "tile_log") e->tile_log = v;
            else if (k == "grid") e->grid = v;
            else if (k == "order") e->order = v;
            else if (k == "serial") e->serial = v;
            else return false;
        } while (eat(','));
        return eat('}') && e->valid();
    }
    bool file(Table* t) {
        bool fmt = false, ver = false, ents = false;
        if (!eat('{')) return false;
        do {
            std::string k;
            if (!str(&k) || !eat(':')) return false;
            if (k == "format") {
                std::string v;
                if (!str(&v) || v != "mrdft-tune") return false;
                fmt = true;
            } else if (k == "version") {
                long v = 0;
                if (!integer(&v) || v != MRDFT_TUNE_CACHE_VERSION) return false;
                ver = true;
            } else if (k == "entries") {
                if (!eat('{')) return false;
                if (!eat('}')) {
                    do {
                        std::string key;
                        Entry e;
                        if (!str(&key) || !key_ok(key.c_str()) || !eat(':') || !entry(&e)) return false;
                        (*t)[key] = e;
                    } while (eat(','));
                    if (!eat('}')) return false;
                }
                ents = true;
            } else {
                return false;
            }
        } while (eat(','));
        if (!eat('}')) return false;
        ws();
        return i == s.size() && fmt && ver && ents;
    }
};

// The file's entries, or an empty table if it is missing or not accepted.
Table read_table(const char* path) {
    Table t;
    FILE* f = std::fopen(path, "rb");
    if (!f) return t;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) {
        text.append(buf, n);
        if (text.size() > (64u << 20)) {          // far beyond any real cache: not ours
            std::fclose(f);
            return Table();
        }
    }
    std::fclose(f);
    Reader r(text);
    if (!r.file(&t)) return Table();
    return t;
}

bool write_table(const char* path, const Table& t) {
    std::string out = "{\"format\": \"mrdft-tune\", \"version\": " + std::to_string(MRDFT_TUNE_CACHE_VERSION) +
                      ", \"entries\": {";
    bool first = true;
    for (const auto& kv : t) {
        char line[256];
        std::snprintf(line, sizeof(line), "{\"tile_log\": %ld, \"grid\": %ld, \"order\": %ld, \"serial\": %ld}",
                      kv.second.tile_log, kv.second.grid, kv.second.order, kv.second.serial);
        out += (first ? "\n  \"" : ",\n  \"") + kv.first + "\": " + line;
        first = false;
    }
    out += "\n}}\n";
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return false;
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return false;
    }
    return true;
}

}  // namespace

extern "C" {

int mrdft_tune_cache_lookup(const char* path, const char* key, int* tile_log, int* grid, int* order, int* serial) {
    if (!path || !tile_log || !grid || !order || !serial || !key_ok(key)) return -1;
    const Table t = read_table(path);
    const auto it = t.find(key);
    if (it == t.end()) return 0;
    *tile_log = (int)it->second.tile_log;
    *grid = (int)it->second.grid;
    *order = (int)it->second.order;
    *serial = (int)it->second.serial;
    return 1;
}

int mrdft_tune_cache_store(const char* path, const char* key, int tile_log, int grid, int order, int serial) {
    if (!path || !key_ok(key) || tile_log < 0 || grid < 0 || order < 0 || serial < 0) return 1;
    Table t = read_table(path);
    Entry e;
    e.tile_log = tile_log;
    e.grid = grid;
    e.order = order;
    e.serial = serial;
    t[key] = e;
    return write_table(path, t) ? 0 : 3;
}

}  // extern "C"
