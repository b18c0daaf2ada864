"""Write the tuning table the library loads by default (tor_tuning.json beside
libtorgbs.so): wave-tier task sizes of the batched path per (precision, n)
(tor_autotune) and unit depths of the persistent kernel per n
(tor_pserver_autotune), measured on the GPU it runs on.

    python -m paper_1810_00900_amd.tune [--out PATH] [--persistent-only]
"""
import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tor_tuning.json"))
    ap.add_argument("--n-lo", type=int, default=12)
    ap.add_argument("--n-hi", type=int, default=28)
    ap.add_argument("--ps-n-hi", type=int, default=24)
    ap.add_argument("--persistent-only", action="store_true",
                    help="keep the task sizes of the table the library loads; tune only the unit depths")
    args = ap.parse_args()
    if not args.persistent_only:
        os.environ["TOR_TUNE_CACHE"] = ""  # start from the built-in defaults
    sys.path.insert(0, os.path.dirname(HERE))
    import paper_1810_00900_amd as tg
    with tg.Context(0) as ctx:
        for prec in (() if args.persistent_only else ("dd", "f64")):
            print(f"tuning task sizes ({prec}), n = {args.n_lo}..{args.n_hi}", flush=True)
            ctx.autotune(prec, args.n_lo, args.n_hi)
        print(f"tuning persistent unit depths, n = {args.n_lo}..{args.ps_n_hi}", flush=True)
        with tg.PServer(ctx) as srv:
            srv.autotune(args.n_lo, args.ps_n_hi, args.out)
        print("wrote", args.out, flush=True)
        print(open(args.out).read(), flush=True)


if __name__ == "__main__":
    main()
