"""A/B: run bench.py against another build of libcosm.so (argv[1]); the rest of argv goes to bench."""
import os
import sys

sys.path.insert(0, os.getcwd())
import paper_2605_30355_amd.cosm as c  # noqa: E402

c._LIB_PATH = os.path.abspath(sys.argv[1])
sys.argv = ["bench.py"] + sys.argv[2:]
import bench  # noqa: E402

bench.main()
