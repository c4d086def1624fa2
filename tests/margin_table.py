"""Print the parity margins collected with FGL_MARGIN_LOG (tests/gpu_util.py)
as a table, worst mixed-precision margin first.

Usage: python tests/margin_table.py <record.jsonl>
"""
import json
import sys


def main(path: str) -> None:
    recs = [json.loads(line) for line in open(path) if line.strip()]
    order = {"mixed": 0, "fp64": 1, "fp32": 2}
    recs.sort(key=lambda r: (order.get(r["prec"], 3), -r["max_ratio"]))
    print(f"{'case':44s} {'prec':5s} {'rows':>6s} {'max|dlnL|':>10s} "
          f"{'max/tol':>10s} {'p99/tol':>10s}")
    for r in recs:
        print(f"{r['case'][:44]:44s} {r['prec']:5s} {r['rows']:6d} {r['max_abs']:10.3e} "
              f"{r['max_ratio']:10.3e} {r['p99_ratio']:10.3e}")
    for p in ("mixed", "fp64"):
        rs = [r["max_ratio"] for r in recs if r["prec"] == p]
        if rs:
            print(f"# {p}: {len(rs)} cases, largest max|dlnL|/tol = {max(rs):.3e}")


if __name__ == "__main__":
    main(sys.argv[1])
