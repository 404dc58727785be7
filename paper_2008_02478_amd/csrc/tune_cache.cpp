// JSON reader and writer of the schedule cache (see tune_cache.hpp).  The
// reader accepts general JSON syntax (objects, arrays, strings, numbers,
// literals) and keeps only the fields of the documented layout.
#include "tune_cache.hpp"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>
#include <unistd.h>

namespace demag {
namespace {

struct Reader {
  const std::string& s;
  size_t i = 0;
  std::string err;

  explicit Reader(const std::string& text) : s(text) {}

  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  bool bad(const char* what) {
    if (err.empty()) err = std::string(what) + " at offset " + std::to_string(i);
    return false;
  }
  bool lit(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool string(std::string& out) {
    ws();
    if (i >= s.size() || s[i] != '"') return bad("expected a string");
    ++i;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) return bad("bad escape");
        const char e = s[i++];
        switch (e) {
          case '"': case '\\': case '/': c = e; break;
          case 'n': c = '\n'; break;
          case 't': c = '\t'; break;
          case 'r': c = '\r'; break;
          case 'b': c = '\b'; break;
          case 'f': c = '\f'; break;
          case 'u':
            if (i + 4 > s.size()) return bad("bad escape");
            i += 4;
            c = '?';
            break;
          default: return bad("bad escape");
        }
      }
      out.push_back(c);
    }
    if (i >= s.size()) return bad("unterminated string");
    ++i;
    return true;
  }
  bool number(double& v) {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    v = std::strtod(b, &e);
    if (e == b) return bad("expected a number");
    i += (size_t)(e - b);
    return true;
  }
  // skips any JSON value
  bool skip() {
    ws();
    if (i >= s.size()) return bad("unexpected end");
    const char c = s[i];
    if (c == '"') {
      std::string t;
      return string(t);
    }
    if (c == '{' || c == '[') {
      const char close = c == '{' ? '}' : ']';
      ++i;
      if (lit(close)) return true;
      do {
        if (c == '{') {
          std::string k;
          if (!string(k) || !lit(':')) return bad("bad object");
        }
        if (!skip()) return false;
      } while (lit(','));
      return lit(close) ? true : bad("bad container");
    }
    for (const char* w : {"true", "false", "null"}) {
      const size_t n = std::char_traits<char>::length(w);
      if (s.compare(i, n, w) == 0) {
        i += n;
        return true;
      }
    }
    double v;
    return number(v);
  }
  bool entry(TuneEntry& e) {
    if (!lit('{')) return bad("expected an entry object");
    if (lit('}')) return true;
    do {
      std::string k;
      if (!string(k) || !lit(':')) return bad("bad entry");
      if (k == "yg" || k == "kw" || k == "radix" || k == "zsep" || k == "x_us" || k == "mid_us") {
        double v;
        if (!number(v)) return false;
        if (k == "yg") e.yg = (int)v;
        else if (k == "zsep") e.zsep = (int)v;
        else if (k == "kw") e.kw = (int)v;
        else if (k == "radix") e.radix = (int)v;
        else if (k == "x_us") e.x_us = v;
        else e.mid_us = v;
      } else if (!skip()) {
        return false;
      }
    } while (lit(','));
    return lit('}') ? true : bad("bad entry");
  }
};

}  // namespace

bool tune_cache_parse(const std::string& text, TuneMap& out, std::string& err) {
  Reader r(text);
  out.clear();
  bool fmt = false;
  if (!r.lit('{')) {
    err = "schedule cache: not a JSON object";
    return false;
  }
  if (!r.lit('}')) {
    do {
      std::string k;
      if (!r.string(k) || !r.lit(':')) {
        err = "schedule cache: " + r.err;
        return false;
      }
      if (k == "format") {
        std::string f;
        if (!r.string(f)) {
          err = "schedule cache: " + r.err;
          return false;
        }
        fmt = (f == "demag-schedule-cache/1");
      } else if (k == "entries") {
        if (!r.lit('{')) {
          err = "schedule cache: entries must be an object";
          return false;
        }
        if (!r.lit('}')) {
          do {
            std::string key;
            TuneEntry e;
            if (!r.string(key) || !r.lit(':') || !r.entry(e)) {
              err = "schedule cache: " + r.err;
              return false;
            }
            out[key] = e;
          } while (r.lit(','));
          if (!r.lit('}')) {
            err = "schedule cache: unterminated entries";
            return false;
          }
        }
      } else if (!r.skip()) {
        err = "schedule cache: " + r.err;
        return false;
      }
    } while (r.lit(','));
    if (!r.lit('}')) {
      err = "schedule cache: unterminated object";
      return false;
    }
  }
  r.ws();
  if (r.i != text.size()) {
    err = "schedule cache: trailing data";
    return false;
  }
  if (!fmt) {
    err = "schedule cache: missing or unknown \"format\"";
    return false;
  }
  return true;
}

bool tune_cache_read(const std::string& path, TuneMap& out, std::string& err) {
  out.clear();
  std::ifstream f(path, std::ios::binary);
  if (!f) {
    if (access(path.c_str(), F_OK) != 0) return true;   // no cache yet
    err = "schedule cache: cannot read " + path;
    return false;
  }
  std::stringstream ss;
  ss << f.rdbuf();
  return tune_cache_parse(ss.str(), out, err);
}

static std::string quote(const std::string& k) {
  std::string o = "\"";
  for (char c : k) {
    if (c == '"' || c == '\\') o.push_back('\\');
    o.push_back(c);
  }
  return o + "\"";
}

bool tune_cache_write(const std::string& path, const TuneMap& m, std::string& err) {
  std::string text = "{\n  \"format\": \"demag-schedule-cache/1\",\n  \"entries\": {";
  bool first = true;
  char buf[256];
  for (const auto& kv : m) {
    const TuneEntry& e = kv.second;
    std::snprintf(buf, sizeof buf,
                  "{\"yg\": %d, \"kw\": %d, \"radix\": %d, \"zsep\": %d, \"x_us\": %.3f, \"mid_us\": %.3f}", e.yg,
                  e.kw, e.radix, e.zsep, e.x_us, e.mid_us);
    text += first ? "\n    " : ",\n    ";
    text += quote(kv.first) + ": " + buf;
    first = false;
  }
  text += first ? "}\n}\n" : "\n  }\n}\n";
  const std::string tmp = path + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream f(tmp, std::ios::binary | std::ios::trunc);
    if (!f) {
      err = "schedule cache: cannot write " + tmp;
      return false;
    }
    f << text;
    if (!f.good()) {
      err = "schedule cache: write failed for " + tmp;
      return false;
    }
  }
  if (std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    err = "schedule cache: cannot replace " + path;
    return false;
  }
  return true;
}

}  // namespace demag
