// Sanitizer driver of the C-ABI's host-only entry points.  Reads hierarchies
// from stdin, one per line:
//   x0 y0 h0 ratio aspect npatches  (level n ox oy) x npatches
// and prints, per hierarchy, td_hierarchy_check's status, then
// td_plan_check's status and workspace bytes for FP32 and FP64.
#include <cstdio>
#include <vector>

#include "thindisk.h"

int main()
{
    double x0, y0, h0, aspect;
    int ratio, np;
    while (std::scanf("%lf %lf %lf %d %lf %d", &x0, &y0, &h0, &ratio, &aspect, &np) == 6) {
        if (np < 0 || np > 64) return 2;
        std::vector<td_patch> p((size_t)np);
        for (int k = 0; k < np; ++k)
            if (std::scanf("%d %d %d %d", &p[k].level, &p[k].n, &p[k].ox, &p[k].oy) != 4) return 2;
        td_hierarchy h{x0, y0, h0, ratio, np, p.data(), aspect};
        const int chk = td_hierarchy_check(&h);
        size_t ws32 = 0, ws64 = 0;
        const int s32 = td_plan_check(&h, TD_F32, &ws32);
        const int s64 = td_plan_check(&h, TD_F64, &ws64);
        std::printf("%d %d %zu %d %zu\n", chk, s32, ws32, s64, ws64);
    }
    return 0;
}
