// A small JSON reader (objects, arrays, strings, numbers, literals) for the
// wisdom records and the capture headers.  Internal to libkl.
#pragma once

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

namespace kl {


struct JVal {
    enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal *get(const char *key) const
    {
        for (auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char *p, *end;
    bool ok = true;
    void ws()
    {
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
    }
    bool lit(const char *s)
    {
        const size_t n = strlen(s);
        if ((size_t)(end - p) >= n && !strncmp(p, s, n)) {
            p += n;
            return true;
        }
        return false;
    }
    bool string(std::string &out)
    {
        if (p >= end || *p != '"') return false;
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= end) return false;
                switch (*p) {
                case 'n': out += '\n'; break;
                case 't': out += '\t'; break;
                case 'r': out += '\r'; break;
                case 'b': out += '\b'; break;
                case 'f': out += '\f'; break;
                case 'u':
                    if (end - p < 5) return false;
                    out += '?';
                    p += 4;
                    break;
                default: out += *p;
                }
                ++p;
            } else {
                out += *p++;
            }
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool value(JVal &v, int depth)
    {
        if (depth > 16) return false;
        ws();
        if (p >= end) return false;
        if (*p == '{') {
            v.kind = JVal::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') {
                ++p;
                return true;
            }
            for (;;) {
                ws();
                std::string key;
                if (!string(key)) return false;
                ws();
                if (p >= end || *p != ':') return false;
                ++p;
                JVal child;
                if (!value(child, depth + 1)) return false;
                v.obj.emplace_back(std::move(key), std::move(child));
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == '}') {
                    ++p;
                    return true;
                }
                return false;
            }
        }
        if (*p == '[') {
            v.kind = JVal::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') {
                ++p;
                return true;
            }
            for (;;) {
                JVal child;
                if (!value(child, depth + 1)) return false;
                v.arr.push_back(std::move(child));
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == ']') {
                    ++p;
                    return true;
                }
                return false;
            }
        }
        if (*p == '"') {
            v.kind = JVal::STR;
            return string(v.str);
        }
        if (lit("true")) {
            v.kind = JVal::BOOL;
            v.b = true;
            return true;
        }
        if (lit("false")) {
            v.kind = JVal::BOOL;
            return true;
        }
        if (lit("null")) return true;
        char *q = nullptr;
        std::string tmp(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
        v.num = strtod(tmp.c_str(), &q);
        if (q == tmp.c_str()) return false;
        v.kind = JVal::NUM;
        p += (q - tmp.c_str());
        return true;
    }
};

inline bool parse_json(const std::string &s, JVal &out)
{
    JParser ps{s.data(), s.data() + s.size()};
    if (!ps.value(out, 0)) return false;
    ps.ws();
    return ps.p == ps.end;
}

inline std::string json_escape(const std::string &s)
{
    std::string o;
    for (char c : s) {
        if (c == '"' || c == '\\') {
            o += '\\';
            o += c;
        } else if ((unsigned char)c < 0x20) {
            o += ' ';
        } else {
            o += c;
        }
    }
    return o;
}

}  // namespace kl
