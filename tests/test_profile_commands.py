"""Every bench.py command recorded in profiles/ parses with bench.py's
current arguments, so each summary names a command that still runs."""
import glob
import os
import re
import shlex

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def recorded_arg_lists():
    found = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*"))):
        with open(path) as f:
            for line in f:
                # "`<args>` = `--profile-leg ...`" in the counter notes
                for m in re.finditer(r"`<args>` = `([^`]*)`", line):
                    found.append((path, shlex.split(m.group(1))))
                for m in re.finditer(r"python3?\s+\S*bench\.py([^`\"'\n]*)", line):
                    args = [a for a in shlex.split(m.group(1)) if a != "<args>"]
                    if args:
                        found.append((path, args))
    return found


def test_recorded_commands_parse():
    lists = recorded_arg_lists()
    files = {os.path.basename(p) for p, _ in lists}
    # every kernel-statistics and counter summary records its command
    for path in glob.glob(os.path.join(ROOT, "profiles", "*")):
        assert os.path.basename(path) in files, path
    parser = bench.build_parser()
    for path, args in lists:
        ns = parser.parse_args(args)
        assert ns.profile_leg is not None, (path, args)
