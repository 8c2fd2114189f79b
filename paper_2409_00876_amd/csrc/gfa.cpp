// GFA v1 reader: variation graph text -> the lean structure the layout reads.
//
// The layout of Alg. 1 reads only the paths and the node lengths of a graph;
// the GPU kernel of Section "CUDA Kernel for Pangenome Graph Layout" keeps a
// lean copy of exactly that (node lengths, path step lists with orientation),
// and the experiments of Section "Experiment Setup" load the human pangenome
// graphs from their GFA/ODGI files.  This file turns GFA 1.0/1.1 text into
// that structure: S lines give node lengths, P lines (GFA 1.0) and W lines
// (GFA 1.1) give the paths with their orientation, every other record (links,
// containments, jumps, headers, comments) is skipped.  Host code only; it does
// none of the method's arithmetic.
//
// Node ids: segment k of the file (in S-line order) becomes node k.  Path p is
// the p-th P or W line.  A path may name segments whose S line comes later.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pgsgd.h"
#include "device.h"
#include "internal.h"

using namespace pgsgd;

struct pgsgd_gfa {
  // provisional segment index (order of first mention) -> data
  std::vector<uint64_t> seg_len;      // 0 = no S line yet
  std::vector<int64_t> seg_sline;     // S-line ordinal, -1 = not defined yet
  std::vector<uint64_t> seg_name_off; // into seg_names (provisional order)
  std::string seg_names;
  std::unordered_map<std::string, uint32_t> by_name;
  std::vector<uint32_t> by_number;    // decimal names "1".."N": number -> provisional index + 1
  uint32_t n_slines = 0;
  // paths
  std::vector<uint64_t> path_off{0};
  std::vector<uint32_t> step;         // provisional index | reverse << 31
  std::string path_names;
  std::vector<uint64_t> path_name_off{0};
  std::unordered_map<std::string, uint32_t> path_by_name;
  uint64_t n_links = 0;
  // final arrays (after finish())
  std::vector<uint32_t> node_len;
  std::string node_names;
  std::vector<uint64_t> node_name_off;
};

namespace {

constexpr uint32_t kMaxNodes = 1u << 31;
constexpr uint64_t kMaxGfaSteps = 1ull << 40;

struct Reader {
  pgsgd_gfa* G;
  uint64_t line = 0;
  std::string err;
  pgsgd_status code = PGSGD_OK;

  bool bad(pgsgd_status c, const std::string& msg) {
    code = c;
    err = "GFA line " + std::to_string(line) + ": " + msg;
    return false;
  }

  // Index of segment `name` (created on first mention).  Decimal names
  // without a leading zero are kept in a direct table while the numbers stay
  // dense; every other name, and a number first seen far beyond the table,
  // goes to the hash map.  A name is created in exactly one of the two.
  bool segment(const char* name, size_t len, uint32_t* out) {
    if (len == 0) return bad(PGSGD_ERR_INVALID_ARG, "empty segment name");
    uint64_t num = 0;
    bool numeric = len <= 10 && !(name[0] == '0' && len > 1);
    for (size_t k = 0; numeric && k < len; ++k) {
      if (name[k] < '0' || name[k] > '9') numeric = false;
      else num = num * 10 + (uint64_t)(name[k] - '0');
    }
    if (numeric && num < G->by_number.size() && G->by_number[num]) {
      *out = G->by_number[num] - 1;
      return true;
    }
    std::string key(name, len);
    if (!G->by_name.empty()) {
      auto it = G->by_name.find(key);
      if (it != G->by_name.end()) {
        *out = it->second;
        return true;
      }
    }
    if (!add_segment(name, len, out)) return false;
    if (numeric && num <= 64ull * (G->seg_len.size() + (1u << 20))) {
      if (num >= G->by_number.size()) G->by_number.resize(std::max<uint64_t>(num + 1, 2 * G->by_number.size()), 0);
      G->by_number[num] = *out + 1;
    } else {
      G->by_name.emplace(std::move(key), *out);
    }
    return true;
  }

  bool add_segment(const char* name, size_t len, uint32_t* out) {
    if (G->seg_len.size() + 1 >= kMaxNodes) return bad(PGSGD_ERR_RANGE, "2^31 or more segments");
    *out = (uint32_t)G->seg_len.size();
    G->seg_len.push_back(0);
    G->seg_sline.push_back(-1);
    G->seg_name_off.push_back(G->seg_names.size());
    G->seg_names.append(name, len);
    G->seg_names.push_back('\0');
    return true;
  }

  static bool parse_u64(const char* s, size_t len, uint64_t* v) {
    if (len == 0 || len > 19) return false;
    uint64_t x = 0;
    for (size_t k = 0; k < len; ++k) {
      if (s[k] < '0' || s[k] > '9') return false;
      x = x * 10 + (uint64_t)(s[k] - '0');
    }
    *v = x;
    return true;
  }

  // Splits a line into tab-separated fields (pointer, length).
  static void fields(const char* s, size_t n, std::vector<std::pair<const char*, size_t>>& f) {
    f.clear();
    size_t b = 0;
    for (size_t k = 0; k <= n; ++k)
      if (k == n || s[k] == '\t') {
        f.emplace_back(s + b, k - b);
        b = k + 1;
      }
  }

  bool s_line(const std::vector<std::pair<const char*, size_t>>& f) {
    if (f.size() < 3) return bad(PGSGD_ERR_INVALID_ARG, "S line needs a name and a sequence");
    uint32_t idx;
    if (!segment(f[1].first, f[1].second, &idx)) return false;
    if (G->seg_sline[idx] >= 0)
      return bad(PGSGD_ERR_INVALID_ARG, "segment '" + std::string(f[1].first, f[1].second) + "' defined twice");
    const bool star = f[2].second == 1 && f[2].first[0] == '*';
    uint64_t len = star ? 0 : f[2].second;
    bool have_ln = false;
    for (size_t k = 3; k < f.size(); ++k) {
      if (f[k].second >= 5 && std::memcmp(f[k].first, "LN:i:", 5) == 0) {
        uint64_t v;
        if (!parse_u64(f[k].first + 5, f[k].second - 5, &v)) return bad(PGSGD_ERR_INVALID_ARG, "bad LN tag");
        if (!star && v != len)
          return bad(PGSGD_ERR_INVALID_ARG, "LN:i:" + std::to_string(v) + " disagrees with the sequence length " +
                                                std::to_string(len));
        len = v;
        have_ln = true;
      }
    }
    if (star && !have_ln)
      return bad(PGSGD_ERR_INVALID_ARG, "segment '" + std::string(f[1].first, f[1].second) +
                                            "' has no sequence and no LN tag: its length is unknown");
    if (len == 0) return bad(PGSGD_ERR_INVALID_ARG, "segment of length 0");
    if (len >= (1ull << 32)) return bad(PGSGD_ERR_RANGE, "segment longer than 2^32 - 1 nt");
    G->seg_len[idx] = len;
    G->seg_sline[idx] = G->n_slines++;
    return true;
  }

  bool add_step(uint32_t idx, bool rev) {
    if (G->step.size() >= kMaxGfaSteps) return bad(PGSGD_ERR_RANGE, "2^40 or more path steps");
    G->step.push_back(idx | (rev ? kRevBit : 0u));
    return true;
  }

  bool end_path(const std::string& name) {
    const uint64_t n = G->step.size() - G->path_off.back();
    if (n >= (1ull << 32)) return bad(PGSGD_ERR_RANGE, "path '" + name + "' has 2^32 or more steps");
    if (!G->path_by_name.emplace(name, (uint32_t)(G->path_off.size() - 1)).second)
      return bad(PGSGD_ERR_INVALID_ARG, "path name '" + name + "' used twice");
    if (G->path_off.size() > (1u << 20)) return bad(PGSGD_ERR_RANGE, "more than 2^20 paths");
    G->path_off.push_back(G->step.size());
    G->path_names += name;
    G->path_names.push_back('\0');
    G->path_name_off.push_back(G->path_names.size());
    return true;
  }

  // P <name> <seg><+|->,<seg><+|->,... <overlaps>
  bool p_line(const std::vector<std::pair<const char*, size_t>>& f) {
    if (f.size() < 3) return bad(PGSGD_ERR_INVALID_ARG, "P line needs a name and a segment list");
    std::string name(f[1].first, f[1].second);
    const char* s = f[2].first;
    const size_t n = f[2].second;
    if (!(n == 1 && s[0] == '*')) {
      size_t b = 0;
      for (size_t k = 0; k <= n; ++k)
        if (k == n || s[k] == ',') {
          if (k == b) return bad(PGSGD_ERR_INVALID_ARG, "empty step in P line '" + name + "'");
          const char o = s[k - 1];
          if (o != '+' && o != '-')
            return bad(PGSGD_ERR_INVALID_ARG, "step without orientation in P line '" + name + "'");
          uint32_t idx;
          if (!segment(s + b, k - 1 - b, &idx) || !add_step(idx, o == '-')) return false;
          b = k + 1;
        }
    }
    return end_path(name);
  }

  // W <sample> <haplotype> <sequence id> <start> <end> <walk: (>|<)seg ...>
  bool w_line(const std::vector<std::pair<const char*, size_t>>& f) {
    if (f.size() < 7) return bad(PGSGD_ERR_INVALID_ARG, "W line needs 6 fields");
    std::string name = std::string(f[1].first, f[1].second) + "#" + std::string(f[2].first, f[2].second) + "#" +
                       std::string(f[3].first, f[3].second);
    const bool has_range = !(f[4].second == 1 && f[4].first[0] == '*');
    if (has_range) name += ":" + std::string(f[4].first, f[4].second) + "-" + std::string(f[5].first, f[5].second);
    const char* s = f[6].first;
    const size_t n = f[6].second;
    if (!(n == 1 && s[0] == '*')) {
      if (n == 0 || (s[0] != '>' && s[0] != '<'))
        return bad(PGSGD_ERR_INVALID_ARG, "walk of W line '" + name + "' must start with '>' or '<'");
      size_t b = 0;
      for (size_t k = 1; k <= n; ++k)
        if (k == n || s[k] == '>' || s[k] == '<') {
          uint32_t idx;
          if (!segment(s + b + 1, k - b - 1, &idx) || !add_step(idx, s[b] == '<')) return false;
          b = k;
        }
    }
    return end_path(name);
  }

  bool line_text(const char* s, size_t n, std::vector<std::pair<const char*, size_t>>& f) {
    ++line;
    if (n && s[n - 1] == '\r') --n;
    if (n == 0 || s[0] == '#') return true;
    if (n >= 2 && s[1] != '\t') return bad(PGSGD_ERR_INVALID_ARG, "record type must be one letter and a tab");
    switch (s[0]) {
      case 'H': {
        fields(s, n, f);
        for (size_t k = 1; k < f.size(); ++k)
          if (f[k].second >= 6 && std::memcmp(f[k].first, "VN:Z:", 5) == 0 && f[k].first[5] == '2')
            return bad(PGSGD_ERR_UNSUPPORTED, "GFA 2 is not supported (GFA 1.0 and 1.1 are)");
        return true;
      }
      case 'S': fields(s, n, f); return s_line(f);
      case 'P': fields(s, n, f); return p_line(f);
      case 'W': fields(s, n, f); return w_line(f);
      case 'L': ++G->n_links; return true;
      default: return true;  // containments, jumps, other record types: not used by the layout
    }
  }

  // Renumbers segments in S-line order and checks that every path step names a defined segment.
  bool finish() {
    const size_t n = G->seg_len.size();
    std::vector<uint32_t> final_id(n);
    for (size_t k = 0; k < n; ++k) {
      if (G->seg_sline[k] < 0) {
        line = 0;
        code = PGSGD_ERR_INVALID_ARG;
        err = "GFA: a path visits segment '" + std::string(G->seg_names.c_str() + G->seg_name_off[k]) +
              "', which has no S line";
        return false;
      }
      final_id[k] = (uint32_t)G->seg_sline[k];
    }
    for (uint32_t& v : G->step) v = final_id[v & kNodeMask] | (v & kRevBit);
    G->node_len.assign(n, 0);
    std::vector<uint64_t> name_len(n);
    for (size_t k = 0; k < n; ++k) {
      G->node_len[final_id[k]] = (uint32_t)G->seg_len[k];
      name_len[final_id[k]] = std::strlen(G->seg_names.c_str() + G->seg_name_off[k]) + 1;
    }
    G->node_name_off.assign(n + 1, 0);
    for (size_t k = 0; k < n; ++k) G->node_name_off[k + 1] = G->node_name_off[k] + name_len[k];
    G->node_names.assign(G->node_name_off[n], '\0');
    for (size_t k = 0; k < n; ++k)
      std::memcpy(&G->node_names[G->node_name_off[final_id[k]]], G->seg_names.c_str() + G->seg_name_off[k],
                  name_len[final_id[k]]);
    // drop the parse-time tables
    std::vector<uint64_t>().swap(G->seg_len);
    std::vector<int64_t>().swap(G->seg_sline);
    std::vector<uint64_t>().swap(G->seg_name_off);
    std::string().swap(G->seg_names);
    std::unordered_map<std::string, uint32_t>().swap(G->by_name);
    std::vector<uint32_t>().swap(G->by_number);
    return true;
  }
};

pgsgd_status run_reader(pgsgd_gfa* G, Reader& R, pgsgd_gfa** out) {
  if (R.code != PGSGD_OK || !R.finish()) {
    const pgsgd_status c = R.code;
    delete G;
    return set_error(c, "%s", R.err.c_str());
  }
  *out = G;
  return clear_error();
}

}  // namespace

extern "C" {

pgsgd_status pgsgd_gfa_parse(const char* text, uint64_t n_bytes, pgsgd_gfa** out) {
  if (!out) return set_error(PGSGD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!text && n_bytes) return set_error(PGSGD_ERR_INVALID_ARG, "text is NULL");
  pgsgd_gfa* G = new (std::nothrow) pgsgd_gfa();
  if (!G) return set_error(PGSGD_ERR_OOM, "host allocation failed");
  Reader R{G};
  std::vector<std::pair<const char*, size_t>> f;
  try {
    uint64_t b = 0;
    while (b < n_bytes) {
      const void* nl = std::memchr(text + b, '\n', n_bytes - b);
      const uint64_t e = nl ? (uint64_t)((const char*)nl - text) : n_bytes;
      if (!R.line_text(text + b, e - b, f)) break;
      b = e + 1;
    }
  } catch (const std::bad_alloc&) {
    delete G;
    return set_error(PGSGD_ERR_OOM, "host allocation failed while reading GFA");
  }
  return run_reader(G, R, out);
}

pgsgd_status pgsgd_gfa_read(const char* filename, pgsgd_gfa** out) {
  if (!out) return set_error(PGSGD_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!filename) return set_error(PGSGD_ERR_INVALID_ARG, "filename is NULL");
  FILE* fp = std::fopen(filename, "rb");
  if (!fp) return set_error(PGSGD_ERR_INVALID_ARG, "cannot open '%s': %s", filename, std::strerror(errno));
  pgsgd_gfa* G = new (std::nothrow) pgsgd_gfa();
  if (!G) {
    std::fclose(fp);
    return set_error(PGSGD_ERR_OOM, "host allocation failed");
  }
  Reader R{G};
  std::vector<std::pair<const char*, size_t>> f;
  char* buf = nullptr;
  size_t cap = 0;
  bool io_error = false;
  try {
    for (;;) {
      errno = 0;
      const ssize_t n = getline(&buf, &cap, fp);
      if (n < 0) {
        io_error = std::ferror(fp) != 0;
        break;
      }
      size_t len = (size_t)n;
      if (len && buf[len - 1] == '\n') --len;
      if (!R.line_text(buf, len, f)) break;
    }
  } catch (const std::bad_alloc&) {
    std::free(buf);
    std::fclose(fp);
    delete G;
    return set_error(PGSGD_ERR_OOM, "host allocation failed while reading '%s'", filename);
  }
  std::free(buf);
  std::fclose(fp);
  if (io_error && R.code == PGSGD_OK) {
    delete G;
    return set_error(PGSGD_ERR_INVALID_ARG, "read error on '%s'", filename);
  }
  return run_reader(G, R, out);
}

pgsgd_status pgsgd_gfa_get_view(const pgsgd_gfa* G, pgsgd_gfa_view* out) {
  if (!G || !out) return set_error(PGSGD_ERR_INVALID_ARG, "NULL argument");
  out->n_nodes = (uint32_t)G->node_len.size();
  out->n_paths = (uint32_t)(G->path_off.size() - 1);
  out->n_steps = G->step.size();
  out->n_links = G->n_links;
  out->node_len = G->node_len.data();
  out->path_offsets = G->path_off.data();
  out->step_node = G->step.data();
  out->node_names = G->node_names.data();
  out->node_name_offsets = G->node_name_off.data();
  out->path_names = G->path_names.data();
  out->path_name_offsets = G->path_name_off.data();
  return clear_error();
}

void pgsgd_gfa_free(pgsgd_gfa* G) { delete G; }

}  // extern "C"
