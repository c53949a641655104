// io.cpp -- the input and output stages of the search (Fig. 1): the variants
// and the classes read from text files, the saved combinations written to
// one.  Host code only; the formats are described with the entry points in
// fiuncho.h.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fiuncho.h"
#include "internal.hpp"

namespace {

// the whole file, or false
bool slurp(const char *path, std::vector<char> &buf) {
  FILE *f = std::fopen(path, "rb");
  if (!f) return false;
  buf.clear();
  char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof chunk, f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
  const bool ok = !std::ferror(f);
  std::fclose(f);
  return ok;
}

bool is_sep(char c) { return c == ' ' || c == '\t' || c == ',' || c == '\r'; }

int io_error(const char *path, const char *what) {
  return fiuncho::set_error(FIUNCHO_E_IO, (std::string("cannot ") + what + " " + path).c_str());
}

constexpr uint64_t kMaxSamples = (1u << 24) - 1;

}  // namespace

extern "C" {

int fiuncho_read_genotypes(const char *path, uint8_t *genotypes, size_t capacity, uint32_t *snps,
                           uint32_t *samples) {
  if (!path || !snps || !samples) return fiuncho::set_error(FIUNCHO_E_NULL, "a required pointer is NULL");
  std::vector<char> buf;
  if (!slurp(path, buf)) return io_error(path, "read");
  // first pass: the shape and the characters; second pass (genotypes given):
  // the values.  A variant is a line with at least one digit.
  uint64_t rows = 0, cols = 0;
  for (int pass = 0; pass < (genotypes ? 2 : 1); ++pass) {
    if (pass == 1 && capacity < rows * cols)
      return fiuncho::set_error(FIUNCHO_E_SHAPE, "genotype buffer smaller than snps x samples");
    uint64_t row = 0, line = 1;
    size_t i = 0;
    const size_t end = buf.size();
    while (i < end) {
      size_t j = i;
      while (j < end && buf[j] != '\n') ++j;
      if (j > i && buf[i] != '#') {
        uint64_t c = 0;
        uint8_t *dst = pass == 1 ? genotypes + row * cols : nullptr;
        for (size_t p = i; p < j; ++p) {
          const char ch = buf[p];
          if (ch >= '0' && ch <= '2') {
            if (dst) dst[c] = (uint8_t)(ch - '0');
            ++c;
          } else if (!is_sep(ch)) {
            return fiuncho::set_error(FIUNCHO_E_GENOTYPE,
                                      ("genotype other than 0, 1, 2 on line " + std::to_string(line)).c_str());
          }
        }
        if (c > 0) {
          if (pass == 0) {
            if (row == 0) cols = c;
            else if (c != cols)
              return fiuncho::set_error(FIUNCHO_E_SHAPE,
                                        ("variant on line " + std::to_string(line) + " has " +
                                         std::to_string(c) + " samples, the first " + std::to_string(cols))
                                            .c_str());
          }
          ++row;
        }
      }
      i = j + 1;
      ++line;
    }
    if (pass == 0) {
      rows = row;
      if (rows == 0) return fiuncho::set_error(FIUNCHO_E_SHAPE, "no variant in the genotype file");
      if (cols > kMaxSamples) return fiuncho::set_error(FIUNCHO_E_SHAPE, "2^24 samples or more");
      if (rows > 0xFFFFFFFFull) return fiuncho::set_error(FIUNCHO_E_SHAPE, "2^32 variants or more");
    }
  }
  *snps = (uint32_t)rows;
  *samples = (uint32_t)cols;
  return FIUNCHO_OK;
}

int fiuncho_read_phenotype(const char *path, uint8_t *phenotype, size_t capacity, uint32_t *samples) {
  if (!path || !samples) return fiuncho::set_error(FIUNCHO_E_NULL, "a required pointer is NULL");
  std::vector<char> buf;
  if (!slurp(path, buf)) return io_error(path, "read");
  uint64_t count = 0;
  for (int pass = 0; pass < (phenotype ? 2 : 1); ++pass) {
    if (pass == 1 && capacity < count)
      return fiuncho::set_error(FIUNCHO_E_SHAPE, "phenotype buffer smaller than samples");
    uint64_t c = 0, line = 1;
    bool comment = false, line_start = true;
    for (const char ch : buf) {
      if (ch == '\n') {
        ++line;
        comment = false;
        line_start = true;
        continue;
      }
      if (line_start && ch == '#') comment = true;
      line_start = false;
      if (comment) continue;
      if (ch == '0' || ch == '1') {
        if (pass == 1) phenotype[c] = (uint8_t)(ch - '0');
        ++c;
      } else if (!is_sep(ch)) {
        return fiuncho::set_error(FIUNCHO_E_PHENOTYPE,
                                  ("phenotype other than 0 or 1 on line " + std::to_string(line)).c_str());
      }
    }
    if (pass == 0) {
      count = c;
      if (count == 0) return fiuncho::set_error(FIUNCHO_E_SHAPE, "no sample in the phenotype file");
      if (count > kMaxSamples) return fiuncho::set_error(FIUNCHO_E_SHAPE, "2^24 samples or more");
    }
  }
  *samples = (uint32_t)count;
  return FIUNCHO_OK;
}

int fiuncho_write_hits(const char *path, const fiuncho_hit *hits, uint32_t n, int order) {
  if (!path || (!hits && n > 0)) return fiuncho::set_error(FIUNCHO_E_NULL, "a required pointer is NULL");
  if (order < 1 || order > FIUNCHO_MAX_ORDER)
    return fiuncho::set_error(FIUNCHO_E_ORDER, "order outside [1, 8]");
  FILE *f = std::fopen(path, "w");
  if (!f) return io_error(path, "write");
  bool ok = std::fputs("rank", f) >= 0;
  for (int i = 0; i < order; ++i) ok = ok && std::fprintf(f, "\tsnp%d", i + 1) > 0;
  ok = ok && std::fputs("\tmi\tmi32\trel_err\test\n", f) >= 0;
  for (uint32_t h = 0; h < n && ok; ++h) {
    const fiuncho_hit &e = hits[h];
    ok = std::fprintf(f, "%llu", (unsigned long long)e.rank) > 0;
    for (int i = 0; i < order && ok; ++i) ok = std::fprintf(f, "\t%u", e.snp[i]) > 0;
    ok = ok && std::fprintf(f, "\t%.17g\t%.9g\t%.9g\t%.9g\n", e.mi, (double)e.mi32, (double)e.rel_err,
                            (double)e.est) > 0;
  }
  if (std::fclose(f) != 0) ok = false;
  return ok ? FIUNCHO_OK : io_error(path, "write");
}

}  // extern "C"
