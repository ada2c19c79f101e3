// Tuning table and the reader of the autotuner's JSON.
//
// Format (written by paper_1508_07798_amd/autotune.py):
//   {"arch": "gfx950", "entries": [{"scalar": "complex64", "rows": 1024, "nb": 16,
//     "rpt": 4, "nt": 256, "block": 128, ...}, ...]}
// Only the keys scalar, rows, nb, rpt, nt and block of each entry are read; other
// keys (the measured times) are skipped.
#include "tuning.hpp"

#include <dlfcn.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <mutex>
#include <sstream>

#include "../../include/hss.h"
#include "common.hpp"

namespace hss {
namespace {
std::mutex g_mu;
TuneEntry g_tab[4][kTuneClasses];
bool g_explicit = false;  // the table was set by a call: no automatic load afterwards

int class_index(int rows) {
  for (int i = 0; i < kTuneClasses; ++i)
    if (rows <= kTuneClass[i]) return i;
  return -1;
}

int scalar_code(const std::string& s) {
  if (s == "float32") return 0;
  if (s == "float64") return 1;
  if (s == "complex64") return 2;
  if (s == "complex128") return 3;
  return -1;
}

// A small reader for the flat schema above: objects, arrays, strings and integers.
struct Reader {
  const std::string& t;
  size_t i = 0;
  explicit Reader(const std::string& s) : t(s) {}
  [[noreturn]] void bad(const char* what) const {
    throw Error(HSS_EINVAL, std::string("tuning file: ") + what + " at offset " + std::to_string(i));
  }
  void ws() {
    while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  void expect(char c) {
    if (!eat(c)) bad("unexpected character");
  }
  std::string str() {
    expect('"');
    std::string s;
    while (i < t.size() && t[i] != '"') {
      if (t[i] == '\\') ++i;
      if (i < t.size()) s += t[i++];
    }
    expect('"');
    return s;
  }
  double num() {
    ws();
    size_t j = i;
    while (j < t.size() && (std::isdigit((unsigned char)t[j]) || t[j] == '-' || t[j] == '+' || t[j] == '.' ||
                            t[j] == 'e' || t[j] == 'E'))
      ++j;
    if (j == i) bad("number expected");
    const double v = std::strtod(t.substr(i, j - i).c_str(), nullptr);
    i = j;
    return v;
  }
  // skips any value
  void skip() {
    ws();
    if (i >= t.size()) bad("value expected");
    const char c = t[i];
    if (c == '"') {
      str();
    } else if (c == '{') {
      ++i;
      if (eat('}')) return;
      do {
        str();
        expect(':');
        skip();
      } while (eat(','));
      expect('}');
    } else if (c == '[') {
      ++i;
      if (eat(']')) return;
      do skip();
      while (eat(','));
      expect(']');
    } else if (t.compare(i, 4, "true") == 0 || t.compare(i, 4, "null") == 0) {
      i += 4;
    } else if (t.compare(i, 5, "false") == 0) {
      i += 5;
    } else {
      num();
    }
  }
};
}  // namespace

bool tuning_lookup(int scalar, int rows, TuneEntry& e) {
  const int c = class_index(rows);
  if (scalar < 0 || scalar > 3 || c < 0) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  e = g_tab[scalar][c];
  return e.nt > 0 || e.block >= 0;
}

void tuning_set(int scalar, int cls_rows, const TuneEntry& e) {
  const int c = class_index(cls_rows);
  if (scalar < 0 || scalar > 3 || c < 0 || kTuneClass[c] != cls_rows)
    throw Error(HSS_EINVAL, "tuning: unknown scalar or size class " + std::to_string(cls_rows));
  std::lock_guard<std::mutex> lk(g_mu);
  g_tab[scalar][c] = e;
  g_explicit = true;
}

void tuning_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& row : g_tab)
    for (auto& e : row) e = TuneEntry{};
  g_explicit = true;
}

int tuning_load(const std::string& path) {
  std::ifstream f(path);
  if (!f) throw Error(HSS_EINVAL, "cannot read tuning file " + path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Reader r(text);
  std::vector<std::pair<std::pair<int, int>, TuneEntry>> got;
  r.expect('{');
  if (!r.eat('}')) {
    do {
      const std::string key = r.str();
      r.expect(':');
      if (key != "entries") {
        r.skip();
        continue;
      }
      r.expect('[');
      if (r.eat(']')) continue;
      do {
        r.expect('{');
        int scalar = -1, rows = 0;
        TuneEntry e;
        if (!r.eat('}')) {
          do {
            const std::string k = r.str();
            r.expect(':');
            if (k == "scalar") scalar = scalar_code(r.str());
            else if (k == "rows") rows = (int)r.num();
            else if (k == "nb") e.nb = (int)r.num();
            else if (k == "rpt") e.rpt = (int)r.num();
            else if (k == "nt") e.nt = (int)r.num();
            else if (k == "block") e.block = (int)r.num();
            else r.skip();
          } while (r.eat(','));
          r.expect('}');
        }
        const int c = class_index(rows);
        if (scalar < 0 || c < 0 || kTuneClass[c] != rows) r.bad("entry with an unknown scalar or size class");
        got.push_back({{scalar, rows}, e});
      } while (r.eat(','));
      r.expect(']');
    } while (r.eat(','));
    r.expect('}');
  }
  for (auto& g : got) tuning_set(g.first.first, g.first.second, g.second);
  return (int)got.size();
}

void tuning_load_default() {
  static std::once_flag once;
  std::call_once(once, [] {
    {
      std::lock_guard<std::mutex> lk(g_mu);
      if (g_explicit) return;
    }
    std::string path;
    if (const char* env = std::getenv("HSS_TUNING")) {
      path = env;  // empty: no table
    } else {
      Dl_info info;
      if (dladdr((void*)&tuning_load_default, &info) && info.dli_fname) {
        path = info.dli_fname;
        const size_t s = path.rfind('/');
        path = (s == std::string::npos ? std::string(".") : path.substr(0, s)) + "/tuning_gfx950.json";
      }
    }
    if (path.empty()) return;
    std::ifstream probe(path);
    if (!probe) return;
    try {
      tuning_load(path);
    } catch (const Error&) {
      tuning_clear();  // a malformed default file leaves the built-in rules
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_explicit = false;
  });
}

}  // namespace hss
