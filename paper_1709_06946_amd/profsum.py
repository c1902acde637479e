"""Summaries of rocprofv3 output for the library's kernels.

python -m paper_1709_06946_amd.profsum stats DIR      per-kernel time table
python -m paper_1709_06946_amd.profsum pmc DIR         per-kernel mean counters

DIR is the `-d` directory of a `rocprofv3 --kernel-trace --stats` run (files
`*_kernel_stats.csv`) or of a `rocprofv3 --pmc ...` run (files
`*_counter_collection.csv`).  Kernel names are shortened to the function name
and template arguments.
"""
import collections
import csv
import glob
import os
import re
import sys


def short_name(name):
    name = name.strip()
    name = re.sub(r'\(.*$', '', name)            # argument list
    name = re.sub(r'^void ', '', name)
    name = name.replace('pse::', '')
    name = name.replace('HIP_vector_type<double, 2u>', 'double2')
    name = name.replace('HIP_vector_type<float, 2u>', 'float2')
    return name.strip()


def _files(d, suffix):
    return sorted(glob.glob(os.path.join(d, '**', f'*{suffix}'), recursive=True))


def kernel_stats(d):
    """Rows of the kernel statistics: name, calls, total_ms, avg_us, pct."""
    out = collections.OrderedDict()
    for f in _files(d, 'kernel_stats.csv'):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                name = short_name(r['Name'])
                calls = int(r['Calls'])
                tot = float(r['TotalDurationNs'])
                e = out.setdefault(name, [0, 0.0])
                e[0] += calls
                e[1] += tot
    total = sum(v[1] for v in out.values()) or 1.0
    rows = [dict(name=k, calls=v[0], total_ms=v[1] / 1e6, avg_us=v[1] / v[0] / 1e3,
                 pct=100.0 * v[1] / total) for k, v in out.items()]
    return sorted(rows, key=lambda r: -r['total_ms'])


def counters(d):
    """{kernel: {counter: (dispatches, mean value per dispatch)}}."""
    acc = collections.defaultdict(lambda: collections.defaultdict(lambda: [0, 0.0]))
    for f in _files(d, 'counter_collection.csv'):
        with open(f) as fh:
            per = collections.defaultdict(float)     # (dispatch, kernel, counter) -> sum
            for r in csv.DictReader(fh):
                key = (r.get('Dispatch_Id', ''), short_name(r['Kernel_Name']), r['Counter_Name'])
                per[key] += float(r['Counter_Value'])
            for (_, k, c), v in per.items():
                e = acc[k][c]
                e[0] += 1
                e[1] += v
    return {k: {c: (e[0], e[1] / e[0]) for c, e in cs.items()} for k, cs in acc.items()}


_TRAFFIC = re.compile(r'<!-- traffic stage=(\w+) bytes_per_launch=(\d+) sources=([^ ]+) -->')


def recorded_traffic(stage, profile_file):
    """HBM bytes per launch of `stage` recorded in a committed traffic summary,
    or None when the file is missing or any kernel source it names has changed
    since the counters were taken (sources are hashed with sha256)."""
    import hashlib
    if not os.path.exists(profile_file):
        return None
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'csrc')
    for m in _TRAFFIC.finditer(open(profile_file).read()):
        if m.group(1) != stage:
            continue
        for item in m.group(3).split(','):
            name, digest = item.split(':')
            path = os.path.join(csrc, name)
            if not os.path.exists(path):
                return None
            if hashlib.sha256(open(path, 'rb').read()).hexdigest()[:len(digest)] != digest:
                return None
        return float(m.group(2))
    return None


def main(argv):
    if len(argv) != 3 or argv[1] not in ('stats', 'pmc'):
        print(__doc__)
        return 2
    if argv[1] == 'stats':
        rows = kernel_stats(argv[2])
        print('| kernel | calls | total ms | avg us | % |')
        print('|---|---:|---:|---:|---:|')
        for r in rows:
            print(f"| `{r['name']}` | {r['calls']} | {r['total_ms']:.3f} | {r['avg_us']:.2f} "
                  f"| {r['pct']:.1f} |")
    else:
        cs = counters(argv[2])
        names = sorted({c for v in cs.values() for c in v})
        print('| kernel | dispatches | ' + ' | '.join(f'{n} (mean)' for n in names) + ' |')
        print('|---|---:|' + '---:|' * len(names))
        for k in sorted(cs):
            v = cs[k]
            disp = max(e[0] for e in v.values())
            print(f'| `{k}` | {disp} | ' +
                  ' | '.join(f'{v[n][1]:.1f}' if n in v else '' for n in names) + ' |')
    return 0


if __name__ == '__main__':
    sys.exit(main(sys.argv))
