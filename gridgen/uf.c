/* Union-find connectivity test for the synthetic input generator (graph
 * plumbing only: used to reject topology candidates that island the grid). */
#include <stdlib.h>

static int find(int *p, int a) {
  while (p[a] != a) {
    p[a] = p[p[a]];
    a = p[a];
  }
  return a;
}

/* 1 if the graph on n nodes with edges (f[e], t[e]) for alive[e] != 0 is connected. */
int gg_connected(int n, int m, const long long *f, const long long *t, const unsigned char *alive) {
  if (n <= 1) return 1;
  int *p = (int *)malloc(sizeof(int) * 2 * (size_t)n);
  if (!p) return -1;
  int *sz = p + n;
  for (int i = 0; i < n; ++i) {
    p[i] = i;
    sz[i] = 1;
  }
  int comps = n;
  for (int e = 0; e < m && comps > 1; ++e) {
    if (alive && !alive[e]) continue;
    int a = find(p, (int)f[e]), b = find(p, (int)t[e]);
    if (a != b) {
      if (sz[a] > sz[b]) {
        int tmp = a;
        a = b;
        b = tmp;
      }
      p[a] = b; /* union by size */
      sz[b] += sz[a];
      --comps;
    }
  }
  free(p);
  return comps == 1;
}
