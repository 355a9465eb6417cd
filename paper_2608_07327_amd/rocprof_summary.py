"""Per-kernel summary of rocprofv3 runs of the benchmark: the average duration
of the launches that did work (from a --kernel-trace database), HBM bytes
per launch from a FETCH_SIZE and a WRITE_SIZE counter pass (each scaled by
what the counter reads for the library's 1 GiB streaming copy, which the
benchmark runs), and optionally the MFMA counters of a third pass.

    python3 -m paper_2608_07327_amd.rocprof_summary TRACE_DB FETCH_CSV WRITE_CSV [MFMA_CSV]
        [--record OUT.json --sources k_sparse.hip,dev_common.hpp --record-filter k_spmm]

Launches that exit at once (iterations issued after the solve stopped) are
left out: a kernel's launches shorter than a fifth of its longest are
dropped (--busy-frac; a larger fraction also leaves out shortened trial
runs, such as the batched kernel's autotuning trials).  MFMA: executed MFMA flops per launch from
SQ_INSTS_VALU_MFMA_MOPS_* (x 512), and the MFMA-busy share of the SIMD
cycles (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE per XCD times the
SIMDs).

--record writes the per-launch HBM bytes of every (kernel, grid) pair whose
name matches --record-filter, keyed "S,T,SL,V,U,W@workgroups" for the block
product (the template arguments of its tile shape) and by the full name
otherwise, with a hash of the listed kernel sources (under the package's
csrc/) so that a reader can tell whether the record still describes the
kernel it is used for.

    python3 -m paper_2608_07327_amd.rocprof_summary --counters A.csv [B.csv ...] [--filter RE]

tabulates instead the mean of every counter (and derived metric) of the
given --pmc passes per (kernel, grid), for the kernels matching --filter."""
import argparse, collections, csv, re, sqlite3, statistics, sys


def counters_table(paths, filt, busy_frac):
    """Mean of each counter over the busy launches of every (kernel, grid)."""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    cols = []
    for path in paths:
        disp = collections.defaultdict(dict)
        meta = {}
        for r in csv.DictReader(open(path)):
            k = re.sub(r'\(.*$', '', r['Kernel_Name']).replace('void ', '').replace('mb::', '')
            if filt and not re.search(filt, k):
                continue
            key = (k, int(r['Dispatch_Id']))
            name = r['Counter_Name']
            disp[key][name] = disp[key].get(name, 0.0) + float(r['Counter_Value'])
            meta[key] = (int(r['Grid_Size']) // max(1, int(r['Workgroup_Size'])),
                         int(r['End_Timestamp']) - int(r['Start_Timestamp']))
            if name not in cols:
                cols.append(name)
        groups = collections.defaultdict(list)
        for key, cs in disp.items():
            groups[(key[0], meta[key][0])].append((meta[key][1], cs))
        for g, xs in groups.items():
            m = max(t for t, _ in xs)
            for t, cs in xs:
                if t >= busy_frac * m:
                    for name, v in cs.items():
                        per[g][name].append(v)
    print("| kernel | grid | " + " | ".join(cols) + " |")
    print("|---|---:|" + "---:|" * len(cols))
    for (k, g), cs in sorted(per.items()):
        vals = [f"{statistics.mean(cs[c]):.4g}" if cs.get(c) else "" for c in cols]
        print(f"| `{k[:70]}` | {g} | " + " | ".join(vals) + " |")


def counters_main(argv=None):
    cp = argparse.ArgumentParser()
    cp.add_argument("--counters", nargs="+", required=True)
    cp.add_argument("--filter", default="")
    cp.add_argument("--busy-frac", type=float, default=0.2)
    ca = cp.parse_args(argv)
    counters_table(ca.counters, ca.filter, ca.busy_frac)


def summary(argv=None):
    """The per-kernel summary (and the counter record) of a trace and two
    counter passes."""
    ap = argparse.ArgumentParser()
    ap.add_argument("db"); ap.add_argument("fetch"); ap.add_argument("write")
    ap.add_argument("mfma", nargs="?")
    ap.add_argument("--filter", default="")
    ap.add_argument("--simds", type=int, default=1024)
    ap.add_argument("--xcds", type=int, default=8)
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--record", default="")
    ap.add_argument("--sources", default="")
    ap.add_argument("--record-filter", default="k_spmm")
    ap.add_argument("--workload", default="")
    ap.add_argument("--busy-frac", type=float, default=0.2,
                    help="launches shorter than this fraction of their kernel's (and grid's) "
                         "longest are left out")
    a = ap.parse_args(argv)

    def short(name):
        name = re.sub(r'\(.*$', '', name)
        return name.replace('void ', '').replace('mb::', '')

    con = sqlite3.connect(a.db)
    cur = con.cursor()
    tab = [r[0] for r in cur.execute("select name from sqlite_master where name like 'rocpd_kernel_dispatch%'")][0]
    stab = [r[0] for r in cur.execute("select name from sqlite_master where name like 'rocpd_info_kernel_symbol%'")][0]
    scols = [r[1] for r in cur.execute(f"pragma table_info({stab})")]
    names = {r[0]: r[1] for r in cur.execute(f"select id, {'display_name' if 'display_name' in scols else 'kernel_name'} from {stab}")}
    dcols = [r[1] for r in cur.execute(f"pragma table_info({tab})")]
    has_grid = 'grid_size_x' in dcols and 'workgroup_size_x' in dcols
    dur = collections.defaultdict(list)
    dur_grid = collections.defaultdict(list)   # (kernel, workgroups) -> durations
    q = f"select kernel_id, start, end{', grid_size_x, workgroup_size_x' if has_grid else ''} from {tab}"
    for row in cur.execute(q):
        kid, s, e = row[:3]
        dur[short(names.get(kid, str(kid)))].append((e - s) / 1000.0)
        if has_grid and row[4]:
            dur_grid[(short(names.get(kid, str(kid))), row[3] // row[4])].append((e - s) / 1000.0)

    def load(path):
        per = collections.defaultdict(dict)   # (kernel, dispatch) -> counter -> value
        t = {}
        for r in csv.DictReader(open(path)):
            key = (short(r['Kernel_Name']), int(r['Dispatch_Id']))
            per[key][r['Counter_Name']] = per[key].get(r['Counter_Name'], 0.0) + float(r['Counter_Value'])
            t[key] = ((int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1000.0,
                      int(r['Grid_Size']) // max(1, int(r['Workgroup_Size'])))
        out = collections.defaultdict(list)
        for key, cs in per.items():
            out[key[0]].append((cs, t[key][0], t[key][1]))
        return out

    F, Wr = load(a.fetch), load(a.write)
    Mf = load(a.mfma) if a.mfma else {}
    cf = max(c['FETCH_SIZE'] for c, *_ in F['k_stream_copy'])
    cw = max(c['WRITE_SIZE'] for c, *_ in Wr['k_stream_copy'])
    ff, fw = (1 << 30) / (cf * 1024), (1 << 30) / (cw * 1024)
    print(f"calibration (1 GiB k_stream_copy): FETCH_SIZE {cf:.0f} KiB (factor {ff:.3f}), "
          f"WRITE_SIZE {cw:.0f} KiB (factor {fw:.3f})")

    def busy(xs, key):
        if not xs: return []
        m = max(key(x) for x in xs)
        return [x for x in xs if key(x) >= a.busy_frac * m]

    rows = []
    for k in sorted(set(dur) | set(F)):
        if a.filter and not re.search(a.filter, k): continue
        d = busy(dur.get(k, []), lambda x: x)
        f = busy(F.get(k, []), lambda x: x[1])
        w = busy(Wr.get(k, []), lambda x: x[1])
        avg = statistics.mean(d) if d else float('nan')
        fm = statistics.mean(c['FETCH_SIZE'] for c, *_ in f) * 1024 * ff / 1e6 if f else float('nan')
        wm = statistics.mean(c['WRITE_SIZE'] for c, *_ in w) * 1024 * fw / 1e6 if w else float('nan')
        extra = ""
        if Mf.get(k):
            m = busy(Mf[k], lambda x: x[1])
            busyc = sum(c.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) for c, *_ in m)
            gui = sum(c.get('GRBM_GUI_ACTIVE', 0) for c, *_ in m)
            mops = {p: sum(c.get(f'SQ_INSTS_VALU_MFMA_MOPS_{p}', 0) for c, *_ in m) / len(m) for p in ('F64', 'F32', 'BF16')}
            # GRBM_GUI_ACTIVE is counted on every XCD and summed
            util = 100.0 * busyc / (gui / a.xcds * a.simds) if gui else float('nan')
            mt = statistics.mean(t for _, t, _ in m)
            fl = {p: v * 512 for p, v in mops.items() if v}
            extra = f"  MFMA busy {util:5.1f}%" + "".join(f"  {p} {v/1e9:.1f} GFLOP/launch ({v/(mt*1e-6)/1e12:.1f} TFLOP/s)" for p, v in fl.items())
        rows.append((sum(d), k, len(d), avg, fm, wm, extra))
    rows.sort(reverse=True)
    print(f"| kernel | launches | avg us | fetch MB/launch | write MB/launch | MFMA |")
    print("|---|---:|---:|---:|---:|---|")
    for tot, k, nl, avg, fm, wm, extra in rows[:a.top]:
        print(f"| `{k[:80]}` | {nl} | {avg:.2f} | {fm:.1f} | {wm:.1f} | {extra.strip()} |")

    if a.record:
        import hashlib, json, os
        csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
        srcs = [v for v in a.sources.split(",") if v]
        h = hashlib.sha256()
        for f in srcs:
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())

        def rkey(k, g):
            m = re.match(r"k_spmm<BpShape<([\d, ]+)> >", k)
            base = m.group(1).replace(" ", "") if m else k
            return f"{base}@{g}"

        def by_grid(xs):
            out = collections.defaultdict(list)
            for x in xs:
                out[x[2]].append(x)
            return out

        per_shape = {}
        for k in sorted(F):
            if not re.search(a.record_filter, k):
                continue
            fg, wg = by_grid(F[k]), by_grid(Wr.get(k, []))
            for g, fx in fg.items():
                f = busy(fx, lambda x: x[1])
                w = busy(wg.get(g, []), lambda x: x[1])
                if not f or not w:
                    continue
                fb = statistics.mean(c['FETCH_SIZE'] for c, *_ in f) * 1024 * ff
                wb = statistics.mean(c['WRITE_SIZE'] for c, *_ in w) * 1024 * fw
                d = busy(dur_grid.get((k, g), []), lambda x: x)
                per_shape[rkey(k, g)] = {
                    "fetch_bytes": round(fb), "write_bytes": round(wb), "bytes_per_launch": round(fb + wb),
                    "launches": len(f), "avg_us": round(statistics.mean(d), 2) if d else None}
        rec = {"kernel_hash": h.hexdigest()[:16],
               "hashed_sources": [f"paper_2608_07327_amd/csrc/{f}" for f in srcs],
               "workload": a.workload,
               "calibration": {"fetch_factor": ff, "write_factor": fw, "copy_bytes": 1 << 30},
               "per_shape": per_shape}
        with open(a.record, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
        print(f"record: {len(per_shape)} (kernel, grid) entries -> {a.record}")


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if "--counters" in argv:
        counters_main(argv)
    else:
        summary(argv)


if __name__ == "__main__":
    main()
