"""Host check of the cluster-box index arithmetic of the tied order-2 gather
and adjoint kernels (cluster_box.h): tests/cbox_check.cpp walks box_of,
pixel_base, pack_state / packed_base and boxes_fit over random tiles, step
ranges and the window geometries bsf_plan gives, in both direction frames
(Section 1.1's set and the set of Table 1), and checks that every
sub-tap a pixel reads from its LDS box is the window element of that tap, that
every accepted box fits the LDS box and the window (with the spare column of
the pair copies), and that the nine taps per direction are those of the
squared difference operator.  No GPU is used."""
import os
import shutil
import subprocess

import pytest

import paper_1109_5114_amd as bsf

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc is not available")
    exe = str(tmp_path_factory.mktemp("cbox") / "cbox_check")
    subprocess.check_call([HIPCC, "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                           os.path.join(HERE, "cbox_check.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return exe


# (H, W, max_step): the 4096^2 workload's step range, small and ragged images,
# a one-row image, and steps large enough that few tiles fit
GEOMS = [(4096, 4096, 48.0), (37, 53, 9.0), (300, 17, 21.0), (1, 64, 15.0), (129, 2000, 63.0),
         (1024, 1024, 20.0)]
# (frame, tile_w, tile_h, LDS rows): the forward kernel's 16 x 8 tiles with
# 38-row boxes and 16 x 4 tiles with 18-row boxes, the adjoint's 16 x 16 tiles
# with 48-row boxes; in the frame of Table 1's directions the forward's 16 x 8
# tiles and the adjoint's 16 x 16
TILES = [(0, 16, 8, 38), (0, 16, 4, 18), (0, 16, 16, 48), (1, 16, 8, 38), (1, 16, 16, 48)]
DIRS = {0: ((1, 0), (0, 1), (1, 1), (1, -1)), 1: ((2, 1), (1, 2), (1, -2), (2, -1))}


def test_cluster_box_indexing(checker):
    lines = []
    for n, (H, W, ms) in enumerate(GEOMS):
        R_max = int((ms - 1) // 2)
        for frame, tw, th, rows in TILES:
            g = bsf.plan(bsf.Config(dirs=DIRS[frame], order=2, max_step=ms), H, W)
            lines.append("%d %d %d %d %d %d %d %d %d %d %d %d %d" % (frame, H, W, R_max, g.pad_top, g.pad_left,
                                                                     g.win_h, g.win_w, tw, th, rows, 200, 1000 + n))
    p = subprocess.run([checker], input="\n".join(lines) + "\n", capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    words = p.stdout.split()
    assert words[0] == "ok"
    fitting, taps = int(words[1]), int(words[2])
    assert fitting > 500 and taps > 10 ** 8, p.stdout
