// Benchmark-file ingestion (host code only): the text formats in which the
// paper's test instances are distributed (Computational results section: the
// OR-Library bqp sets and the Palubeckis instances), read into the dense
// symmetric int32 matrix that ubqp_problem_create takes.
//
// Both formats are whitespace-separated integers; entries are 1-based (i, j, q)
// triples and each listed value fills q_ij and q_ji.  A pair listed twice must
// carry the same value both times.
//   UBQP_FMT_ORLIB:    K, then K problems, each n, nnz, nnz triples
//   UBQP_FMT_TRIPLETS: one problem: n, nnz, nnz triples
#include "ubqp_internal.h"

#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

struct Reader {
    std::vector<char> buf;  // the file's bytes and a terminating '\0'
    size_t pos = 0, end = 0;
    int64_t tokens = 0;
    char *err;
    int32_t err_len;

    int fail(int code, const char *fmt, ...)
    {
        if (err && err_len > 0) {
            va_list ap;
            va_start(ap, fmt);
            vsnprintf(err, (size_t)err_len, fmt, ap);
            va_end(ap);
        }
        return code;
    }

    // Next integer token; false at the end of the file or on a malformed token.
    bool next(int64_t *v, bool *bad)
    {
        *bad = false;
        while (pos < end && (buf[pos] == ' ' || buf[pos] == '\t' || buf[pos] == '\n' || buf[pos] == '\r'))
            pos++;
        if (pos >= end) return false;
        const char *s = buf.data() + pos;
        char *e = nullptr;
        errno = 0;
        const long long x = strtoll(s, &e, 10);
        const bool sep = *e == '\0' || *e == ' ' || *e == '\t' || *e == '\n' || *e == '\r';
        if (e == s || errno == ERANGE || !sep) {
            *bad = true;
            return false;
        }
        pos += (size_t)(e - s);
        tokens++;
        *v = x;
        return true;
    }
};

}  // namespace

extern "C" int ubqp_read_instance(const char *path, int32_t format, int32_t index, int32_t *count_out, int32_t *n_out,
                                  int32_t *q_host, int64_t q_cap, char *err, int32_t err_len)
{
    Reader r;
    r.err = err;
    r.err_len = err_len;
    if (err && err_len > 0) err[0] = '\0';
    if (!path || !count_out || !n_out) return r.fail(UBQP_EINVAL, "null argument");
    if (format != UBQP_FMT_ORLIB && format != UBQP_FMT_TRIPLETS)
        return r.fail(UBQP_EINVAL, "unknown format %d", format);
    if (index < 0) return r.fail(UBQP_EINVAL, "index %d < 0", index);
    FILE *fp = fopen(path, "rb");
    if (!fp) return r.fail(UBQP_EINVAL, "cannot open %s: %s", path, strerror(errno));
    char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof chunk, fp)) > 0) r.buf.insert(r.buf.end(), chunk, chunk + got);
    const bool rd_err = ferror(fp) != 0;
    fclose(fp);
    if (rd_err) return r.fail(UBQP_EINVAL, "read error on %s", path);
    r.end = r.buf.size();
    r.buf.push_back('\0');  // strtoll stops at it after the last token

    bool bad = false;
    int64_t v = 0;
    auto expect = [&](const char *what) -> int {
        if (r.next(&v, &bad)) return UBQP_OK;
        if (bad) return r.fail(UBQP_EINVAL, "%s: token %lld (%s) is not an integer", path, (long long)r.tokens + 1, what);
        return r.fail(UBQP_EINVAL, "%s: file ends before %s (after %lld tokens)", path, what, (long long)r.tokens);
    };
    int64_t K = 1;
    int rc;
    if (format == UBQP_FMT_ORLIB) {
        if ((rc = expect("the number of problems")) != UBQP_OK) return rc;
        K = v;
        if (K < 1 || K > 1000000) return r.fail(UBQP_EINVAL, "%s: %lld problems", path, (long long)K);
    }
    *count_out = (int32_t)K;
    if (index >= K) return r.fail(UBQP_EINVAL, "%s: index %d, the file holds %lld problems", path, index, (long long)K);
    for (int64_t k = 0; k <= index; k++) {
        if ((rc = expect("n")) != UBQP_OK) return rc;
        const int64_t n = v;
        if ((rc = expect("the number of entries")) != UBQP_OK) return rc;
        const int64_t nnz = v;
        if (n < 1) return r.fail(UBQP_EINVAL, "%s: problem %lld: n = %lld", path, (long long)k, (long long)n);
        if (n > UBQP_MAX_N)
            return r.fail(UBQP_ERANGE, "%s: problem %lld: n = %lld > %d", path, (long long)k, (long long)n, UBQP_MAX_N);
        if (nnz < 0 || nnz > n * n)
            return r.fail(UBQP_EINVAL, "%s: problem %lld: %lld entries for n = %lld", path, (long long)k,
                          (long long)nnz, (long long)n);
        const bool keep = k == index;
        std::vector<uint8_t> seen;
        if (keep) {
            *n_out = (int32_t)n;
            if (q_host) {
                if (q_cap < n * n)
                    return r.fail(UBQP_EINVAL, "%s: problem %lld needs %lld entries, q_cap = %lld", path,
                                  (long long)k, (long long)(n * n), (long long)q_cap);
                memset(q_host, 0, (size_t)(n * n) * sizeof(int32_t));
                seen.assign((size_t)(n * n), 0);
            }
        }
        for (int64_t e = 0; e < nnz; e++) {
            int64_t t[3];
            for (int c = 0; c < 3; c++) {
                if ((rc = expect("an entry")) != UBQP_OK) return rc;
                t[c] = v;
            }
            if (t[0] < 1 || t[0] > n || t[1] < 1 || t[1] > n)
                return r.fail(UBQP_EINVAL, "%s: problem %lld, entry %lld: (%lld, %lld) outside 1..%lld", path,
                              (long long)k, (long long)e + 1, (long long)t[0], (long long)t[1], (long long)n);
            if (t[2] < INT32_MIN || t[2] > INT32_MAX)
                return r.fail(UBQP_ERANGE, "%s: problem %lld, entry %lld: value %lld outside int32", path,
                              (long long)k, (long long)e + 1, (long long)t[2]);
            if (!keep || !q_host) continue;
            const int64_t i = t[0] - 1, j = t[1] - 1;
            const int32_t q = (int32_t)t[2];
            for (int s = 0; s < 2; s++) {
                const int64_t a = s ? j : i, b = s ? i : j;
                uint8_t &m = seen[(size_t)(a * n + b)];
                if (m && q_host[a * n + b] != q)
                    return r.fail(UBQP_EASYM, "%s: problem %lld: (%lld, %lld) listed with %d and %d", path,
                                  (long long)k, (long long)i + 1, (long long)j + 1, q_host[a * n + b], q);
                q_host[a * n + b] = q;
                m = 1;
            }
        }
    }
    return UBQP_OK;
}
