// JSON cache of the autotuner (host code): a small recursive-descent reader
// for the subset the cache uses (objects, strings, numbers; arrays, true,
// false and null are accepted and skipped) and a writer of the same form.
#include "tune_cache.h"

#include <unistd.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>

namespace tufrg {

namespace {

struct Reader {
  const std::string &s;
  size_t i = 0;
  std::string err;

  void ws() {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
  }
  bool expect(char ch) {
    ws();
    if (i < s.size() && s[i] == ch) {
      ++i;
      return true;
    }
    err = std::string("expected '") + ch + "' at offset " + std::to_string(i);
    return false;
  }
  bool string(std::string &out) {
    if (!expect('"')) return false;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      if (s[i] == '\\') {
        if (++i >= s.size()) break;
        const char e = s[i];
        out += e == 'n' ? '\n' : e == 't' ? '\t' : e;  // \" \\ \/ and the rest literally
      } else {
        out += s[i];
      }
      ++i;
    }
    if (i >= s.size()) {
      err = "unterminated string";
      return false;
    }
    ++i;
    return true;
  }
  bool number(double &out) {
    ws();
    const char *b = s.c_str() + i;
    char *e = nullptr;
    out = std::strtod(b, &e);
    if (e == b) {
      err = "expected a number at offset " + std::to_string(i);
      return false;
    }
    i += (size_t)(e - b);
    return true;
  }
  // any value, discarded
  bool skip() {
    ws();
    if (i >= s.size()) {
      err = "unexpected end";
      return false;
    }
    const char ch = s[i];
    if (ch == '"') {
      std::string t;
      return string(t);
    }
    if (ch == '{' || ch == '[') {
      const char close = ch == '{' ? '}' : ']';
      ++i;
      ws();
      if (i < s.size() && s[i] == close) {
        ++i;
        return true;
      }
      for (;;) {
        if (ch == '{') {
          std::string k;
          if (!string(k) || !expect(':')) return false;
        }
        if (!skip()) return false;
        ws();
        if (i < s.size() && s[i] == ',') {
          ++i;
          continue;
        }
        return expect(close);
      }
    }
    for (const char *w : {"true", "false", "null"})
      if (s.compare(i, std::strlen(w), w) == 0) {
        i += std::strlen(w);
        return true;
      }
    double d;
    return number(d);
  }
  // {"key": {"name": number, ...}, ...}
  bool entries(TuneEntries &out) {
    if (!expect('{')) return false;
    ws();
    if (i < s.size() && s[i] == '}') {
      ++i;
      return true;
    }
    for (;;) {
      std::string key;
      if (!string(key) || !expect(':') || !expect('{')) return false;
      auto &m = out[key];
      ws();
      if (i < s.size() && s[i] == '}') {
        ++i;
      } else {
        for (;;) {
          std::string name;
          double v;
          if (!string(name) || !expect(':') || !number(v)) return false;
          m[name] = v;
          ws();
          if (i < s.size() && s[i] == ',') {
            ++i;
            continue;
          }
          if (!expect('}')) return false;
          break;
        }
      }
      ws();
      if (i < s.size() && s[i] == ',') {
        ++i;
        continue;
      }
      return expect('}');
    }
  }
  bool document(TuneEntries &out) {
    if (!expect('{')) return false;
    bool seen = false;
    ws();
    if (i < s.size() && s[i] == '}') {
      ++i;
    } else {
      for (;;) {
        std::string k;
        if (!string(k) || !expect(':')) return false;
        if (k == "entries") {
          if (!entries(out)) return false;
          seen = true;
        } else if (!skip()) {
          return false;
        }
        ws();
        if (i < s.size() && s[i] == ',') {
          ++i;
          continue;
        }
        if (!expect('}')) return false;
        break;
      }
    }
    ws();
    if (i != s.size()) {
      err = "trailing characters after the object";
      return false;
    }
    if (!seen) {
      err = "no \"entries\" object";
      return false;
    }
    return true;
  }
};

std::string quoted(const std::string &k) {
  std::string o = "\"";
  for (char ch : k) {
    if (ch == '"' || ch == '\\') o += '\\';
    o += ch;
  }
  return o + "\"";
}

}  // namespace

bool tune_cache_read(const std::string &path, TuneEntries &out, std::string &err) {
  out.clear();
  std::ifstream f(path, std::ios::binary);
  if (!f) return true;  // no cache yet
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Reader r{text};
  if (!r.document(out)) {
    out.clear();
    err = "tuning cache " + path + " is not a tuning cache (" + r.err + ")";
    return false;
  }
  return true;
}

bool tune_cache_write(const std::string &path, const TuneEntries &entries, std::string &err) {
  const std::string tmp = path + ".tmp." + std::to_string((long long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) {
      err = "cannot write " + tmp;
      return false;
    }
    f << "{\n  \"version\": 1,\n  \"entries\": {";
    bool first = true;
    for (const auto &e : entries) {
      f << (first ? "\n" : ",\n") << "    " << quoted(e.first) << ": {";
      bool f2 = true;
      for (const auto &kv : e.second) {
        char num[64];
        std::snprintf(num, sizeof(num), "%.17g", kv.second);
        f << (f2 ? "" : ", ") << quoted(kv.first) << ": " << num;
        f2 = false;
      }
      f << "}";
      first = false;
    }
    f << (entries.empty() ? "}\n}\n" : "\n  }\n}\n");
    if (!f) {
      err = "cannot write " + tmp;
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    err = "cannot replace " + path;
    return false;
  }
  return true;
}

}  // namespace tufrg
