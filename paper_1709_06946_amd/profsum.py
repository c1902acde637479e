"""Summaries of rocprofv3 output for the library's kernels.

python -m paper_1709_06946_amd.profsum stats DIR      per-kernel time table
python -m paper_1709_06946_amd.profsum pmc DIR         per-kernel mean counters
python -m paper_1709_06946_amd.profsum traffic FETCH WRITE COPY_FETCH COPY_WRITE STAGE
                                                      HBM bytes per launch of one stage

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


# Kernels whose launches make up one stage of the wave-space product.
STAGE_PREFIX = {'fft': ('fft_',), 'kspace': ('kspace_fused', 'kspace_dg3'),
                'spread': ('spread_list', 'spread_deriv'),
                'interp': ('interp_kernel', 'interp_deriv'), 'real': ('real_pair',)}
STAGE_SOURCES = {'fft': ('fft.hip', 'fftreg.h'), 'kspace': ('grid.hip', 'fftreg.h'),
                 'spread': ('grid.hip',), 'interp': ('grid.hip',), 'real': ('real.hip',)}
COPY_BYTES = 2**30


def _copy_counter(d, counter):
    """Mean per dispatch of one counter for the copy kernel of a calibration
    run (the kernel with the largest mean; each dispatch copies 1 GiB)."""
    return max(cs[counter][1] for cs in counters(d).values() if counter in cs)


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, stage):
    """Markdown rows of fetched/written MB per launch, scaled by what the same
    counters read for a 1 GiB device copy, and the stamped total for `stage`
    (bytes per launch, with the sha256 of the sources its kernels come from)."""
    import hashlib
    fscale = COPY_BYTES / (1024 * _copy_counter(copy_fetch_dir, 'FETCH_SIZE'))
    wscale = COPY_BYTES / (1024 * _copy_counter(copy_write_dir, 'WRITE_SIZE'))
    fc, wc = counters(fetch_dir), counters(write_dir)
    rows = []
    for k in set(fc) | set(wc):
        n = max(fc.get(k, {}).get('FETCH_SIZE', (0, 0))[0],
                wc.get(k, {}).get('WRITE_SIZE', (0, 0))[0])
        fb = 1024 * fscale * fc.get(k, {}).get('FETCH_SIZE', (0, 0.0))[1]
        wb = 1024 * wscale * wc.get(k, {}).get('WRITE_SIZE', (0, 0.0))[1]
        rows.append((k, n, fb, wb))
    rows.sort(key=lambda r: -(r[2] + r[3]) * r[1])
    out = [f'Calibration: fetched bytes = {fscale:.3f} x FETCH_SIZE KiB x 1024, '
           f'written bytes = {wscale:.3f} x WRITE_SIZE KiB x 1024 (1 GiB device copy).', '',
           '| kernel | launches | fetched MB | written MB |', '|---|---:|---:|---:|']
    out += [f'| `{k}` | {n} | {fb / 1e6:.1f} | {wb / 1e6:.1f} |' for k, n, fb, wb in rows]
    sel = [r for r in rows if r[0].startswith(STAGE_PREFIX[stage])]
    launches = sum(r[1] for r in sel)
    total = sum((r[2] + r[3]) * r[1] for r in sel) / max(launches, 1)
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), 'csrc')
    srcs = ','.join(f'{f}:' + hashlib.sha256(open(os.path.join(csrc, f), 'rb').read())
                    .hexdigest()[:16] for f in STAGE_SOURCES[stage])
    out += ['', f'Stage `{stage}` (all {", ".join(STAGE_PREFIX[stage])}* launches): '
            f'{total / 1e6:.1f} MB per launch over {launches} launches.', '',
            f'<!-- traffic stage={stage} bytes_per_launch={round(total)} sources={srcs} -->']
    return '\n'.join(out)


def main(argv):
    if len(argv) == 7 and argv[1] == 'traffic':
        print(traffic(*argv[2:7]))
        return 0
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
