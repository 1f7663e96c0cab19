/* Test harness (CPU only): a plain C consumer of the C ABI.  Compiled with
 * gcc against include/dbbc.h and linked with libdbbc.so, it shows that the
 * header is C (no C++ or torch types) and exercises the calls that need no
 * device: version, status strings and argument checks. */
#include <stdio.h>
#include <string.h>

#include "dbbc.h"

int main(void) {
  int fails = 0;
#define CHECK(cond)                                      \
  do {                                                   \
    if (!(cond)) {                                       \
      fprintf(stderr, "failed: %s\n", #cond);            \
      ++fails;                                           \
    }                                                    \
  } while (0)
  CHECK(strlen(dbbc_version()) > 0);
  CHECK(strcmp(dbbc_status_string(DBBC_OK), "ok") == 0 || strlen(dbbc_status_string(DBBC_OK)) > 0);
  CHECK(strlen(dbbc_status_string(DBBC_E_PARSE)) > 0);
  dbbc_graph *g = NULL;
  int32_t u[2] = {0, 1}, v[2] = {0, 1};
  int8_t s[2] = {1, -1};
  CHECK(dbbc_graph_create(0, 2, 2, u, v, s, 0, NULL, NULL, &g) == DBBC_E_INVALID_ARG && g == NULL);
  CHECK(strlen(dbbc_last_error()) > 0);
  CHECK(dbbc_graph_create(2, 2, 2, u, v, s, 0x80u, NULL, NULL, &g) == DBBC_E_INVALID_ARG);
  dbbc_allocator half = {NULL, NULL, NULL};
  CHECK(dbbc_graph_create(2, 2, 2, u, v, s, 0, &half, NULL, &g) == DBBC_E_INVALID_ARG);
  CHECK(dbbc_graph_create_text(NULL, 4, 0, NULL, NULL, &g, NULL) == DBBC_E_INVALID_ARG);
  dbbc_counts c;
  CHECK(dbbc_count(NULL, NULL, &c, NULL) == DBBC_E_INVALID_ARG);
  CHECK(dbbc_count_per_edge(NULL, NULL, NULL, NULL, NULL, NULL) == DBBC_E_INVALID_ARG);
  CHECK(dbbc_count_explicit(NULL, &c, NULL) == DBBC_E_INVALID_ARG);
  dbbc_graph_destroy(NULL);
  printf("%s\n", fails ? "FAIL" : "ok");
  return fails ? 1 : 0;
}
