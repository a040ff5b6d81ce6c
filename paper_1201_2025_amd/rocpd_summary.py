"""Summary of a rocprofv3 results database (the rocpd SQLite file of a kernel trace or of a
--pmc run): per kernel, the dispatch count, the average duration and the sum of every
collected counter over all dispatches and hardware instances.

    python -m paper_1201_2025_amd.rocpd_summary RESULTS.db LABEL

Prints the database's schema instead when the expected columns are missing."""
import re, sqlite3, sys
db, label = sys.argv[1], sys.argv[2]
con = sqlite3.connect(db)
cur = con.cursor()
def cols(v):
    return [r[1] for r in cur.execute("pragma table_info(%s)" % v)]
views = [r[0] for r in cur.execute("select name from sqlite_master where type in ('table','view')")]
out = ["# %s" % label]
if "counters_collection" in views:
    c = cols("counters_collection")
    kn = "kernel_name" if "kernel_name" in c else None
    cn = "counter_name" if "counter_name" in c else None
    val = "value" if "value" in c else None
    if kn and cn and val:
        agg = {}
        for k, n, v in cur.execute("select %s, %s, %s from counters_collection" % (kn, cn, val)):
            k = re.sub(r"\(.*", "", k)[:80]
            agg.setdefault(k, {}).setdefault(n, 0.0)
            agg[k][n] += float(v)
        disp = {}
        if "kernels" in views:
            kc = cols("kernels")
            nm = "kernel_name" if "kernel_name" in kc else "name"
            for k, s, e in cur.execute("select %s, start, end from kernels" % nm):
                k = re.sub(r"\(.*", "", k)[:80]
                d = disp.setdefault(k, [0, 0.0])
                d[0] += 1
                d[1] += (e - s)
        for k in sorted(agg, key=lambda k: -disp.get(k, [0, 0])[1]):
            d = disp.get(k, [0, 0.0])
            out.append("kernel %s | dispatches %d | avg_us %.2f | %s" % (
                k, d[0], d[1] / d[0] / 1e3 if d[0] else 0.0,
                " ".join("%s=%.6g" % kv for kv in sorted(agg[k].items()))))
    else:
        out.append("counters_collection columns: %s" % c)
        for r in cur.execute("select * from counters_collection limit 3"):
            out.append(repr(r))
else:
    out.append("views: %s" % views)
print("\n".join(out))
