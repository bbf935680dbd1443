"""CPU: the launch planner (csrc/kgs_plan.cpp).  The plane-chunk planner of
the z-streaming launches:  A launch runs one workgroup per CU; its
workgroups are dealt to the 8 XCDs in turn, each XCD takes one of 8
contiguous slices of the work items (a tile of one grid by a chunk of its
z-planes) and starts its next item on its first free CU,
an item of L planes taking L + 17 plane-steps.  The planner's estimate is
checked against closed forms (whole rounds) and against a plain simulation
of that rule written here, and its choices against chunks measured on
MI355X (faster: 48 at 224^3 (1.04e11 updates/s against 9.1e10 with 64 and
6.5e10 with 96), 64 at 320^3 and 448^3 in float64; 48 at 224^3 and 96 at
448^3 in float32).  A single grid also tries its equal splits ceil(n / k):
measured, us per 2-step launch, old choice against the equal split,
float64 200^3 172 / 147-152 (32x13 tiles, 64 / 50 planes), 224^3 204 /
197 (16x16, 48 / 45), 448^3 1502-1517 / 1412 (32x13, 96 / 112), float32
448^3 1127-1137 / 1081-1091 (16x32, 96 / 90), 480^3 1461-1491 / 1421
(96 / 120)."""
import heapq
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2502_09537_amd", "csrc")
ITEM = 17
SET = (128, 96, 64, 48, 32, 24, 16, 12, 8)  # the planner's fixed plane chunks


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path_factory.mktemp("plan") / "plan_driver")
    cmd = ["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe,
           os.path.join(ROOT, "tests", "plan", "plan_driver.cpp"),
           os.path.join(CSRC, "kgs_plan.cpp")]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)

    def run(tx, ty, cus, chunk, sizes):
        out = subprocess.run([exe, str(tx), str(ty), str(cus), str(chunk), *map(str, sizes)],
                             check=True, capture_output=True, text=True, timeout=60).stdout.split()
        return (int(out[0]), float(out[1]), tuple(int(v) for v in out[2:5]),
                tuple(int(v) for v in out[5:8]))

    def energy(dim, n, cus):
        out = subprocess.run([exe, "energy", str(dim), str(n), str(cus)], check=True,
                             capture_output=True, text=True, timeout=60).stdout.split()
        return tuple(int(v) for v in out)
    def plan(n, elem_bytes, cus):
        out = subprocess.run([exe, "plan", str(n), str(elem_bytes), str(cus)], check=True,
                             capture_output=True, text=True, timeout=60).stdout.split()
        return tuple(int(v) for v in out)
    run.energy = energy
    run.plan = plan
    return run


def member_chunk(n, chunk):
    """A grid's planes per chunk: the equal split into as many chunks."""
    k = -(-n // chunk)
    return -(-n // k)


def simulate(tx, ty, cus, chunk, sizes):
    """The dealing rule, item by item (each grid with its member_chunk)."""
    lens = []
    for n in sizes:
        tiles = ((n // 2 + tx - 1) // tx) * ((n + ty - 1) // ty)
        cm = member_chunk(n, chunk)
        for z0 in range(0, n, cm):
            lens += [min(cm, n - z0) + ITEM] * tiles
    items = len(lens)
    groups = 8 if cus % 8 == 0 else 1
    per = cus // groups
    q = -(-items // groups)  # contiguous slices of ceil(items / 8), the last ones shorter
    end = 0
    for x in range(groups):
        mine = lens[x * q:(x + 1) * q]
        free = [0] * per
        for L in mine:
            t = heapq.heappop(free) + L
            heapq.heappush(free, t)
            end = max(end, t)
    return end


def test_whole_rounds_closed_form(driver):
    # 256^3, 16x16 tiles: 128 tiles; chunk 128 -> 256 items, one round
    assert driver(16, 16, 256, 128, [256])[1] == 128 + ITEM
    # chunk 64 -> 512 items, two rounds of 64-plane items
    assert driver(16, 16, 256, 64, [256])[1] == 2 * (64 + ITEM)
    # chunk 32 -> 1024 items, four rounds
    assert driver(16, 16, 256, 32, [256])[1] == 4 * (32 + ITEM)
    # fewer items than CUs: the longest item
    assert driver(16, 16, 256, 128, [64])[1] == 64 + ITEM


@pytest.mark.parametrize("tx,ty,cus,chunk,sizes", [
    (16, 16, 256, 96, [224]),            # 294 items: slices of 37, the last 35
    (16, 16, 256, 64, [224]),            # 392 items: slices of 49
    (16, 32, 256, 48, [224, 96, 130]),
    (16, 16, 64, 24, [70, 34, 200, 32]),
    (16, 16, 100, 16, [90, 40]),         # CUs not a multiple of 8: one queue
    (8, 8, 256, 12, [40, 66, 18]),
])
def test_estimate_equals_plain_simulation(driver, tx, ty, cus, chunk, sizes):
    assert driver(tx, ty, cus, chunk, sizes)[1] == simulate(tx, ty, cus, chunk, sizes)


def test_member_chunk_is_the_equal_split():
    # the same number of chunks as the nominal chunk gives, none shorter
    # than the others by more than one plane
    for n in range(2, 600, 3):
        for c in (8, 12, 16, 24, 32, 48, 64, 96, 128):
            m = member_chunk(n, c)
            k = -(-n // c)
            assert m <= c and -(-n // m) == k and n - (k - 1) * m >= m - k


def test_many_items_use_work_over_cus(driver):
    # beyond 16384 items: total steps over the CUs plus one item
    n = 1024
    tiles = (n // 2 // 16) * (n // 16)
    work = tiles * (n + (n // 8) * ITEM)
    assert driver(16, 16, 256, 8, [n])[1] == pytest.approx(work / 256 + 8 + ITEM)


@pytest.mark.parametrize("ty,n,best", [
    (16, 256, 128), (16, 224, 45), (16, 320, 64), (16, 448, 90), (16, 128, 16), (16, 96, 8),
    (32, 256, 64), (32, 224, 45), (32, 448, 90), (32, 512, 128),
])
def test_chosen_chunks(driver, ty, n, best):
    assert driver(16, ty, 256, 0, [n])[0] == best



@pytest.mark.parametrize("tx,ty", [(16, 16), (32, 13), (16, 32)])
def test_single_grid_chunk_is_the_fastest_estimate(driver, tx, ty):
    """One grid: the candidates are the fixed chunks and the equal splits
    ceil(n / k) between 8 and 128; the pick is the longest whose estimate is
    within 1% of every longer one's best (the plain simulation here)."""
    for n in (98, 160, 200, 224, 254, 320, 352, 416, 448, 480):
        assert driver(tx, ty, 256, 0, [n])[0] == planned_chunk(tx, ty, 256, [n]), n


def planned_chunk(tx, ty, cus, sizes):
    """The planner's rule written out: candidates are the fixed chunks and,
    for a single grid, its equal splits ceil(n / k), between 8 and 128,
    scanned from the longest; a shorter one wins only by more than 1%."""
    cands = set(SET)
    if len(sizes) == 1:
        n = sizes[0]
        cands |= {-(-n // k) for k in range(1, n + 1) if 8 <= -(-n // k) <= 128}
    cands = sorted(cands, reverse=True)
    best, best_t = cands[0], simulate(tx, ty, cus, cands[0], sizes)
    for c in cands:
        t = simulate(tx, ty, cus, c, sizes)
        if t < 0.99 * best_t:
            best, best_t = c, t
    return member_chunk(sizes[0], best) if len(sizes) == 1 else best


def test_chosen_chunk_is_the_fastest_estimate(driver):
    sizes = [64, 96, 128, 160, 192, 224, 256, 130, 200, 98]
    best = driver(16, 16, 256, 0, sizes)[0]
    assert best == planned_chunk(16, 16, 256, sizes)
    fixed = min(simulate(16, 16, 256, c, sizes) for c in SET)
    assert simulate(16, 16, 256, best, sizes) <= fixed / 0.99
    # list launches: float32 with its list tile (16x32), float64 with the
    # single-grid tile rule over the whole list
    _, _, l64, l32 = driver(16, 16, 256, 0, sizes)
    assert l32 == (16, 32, driver(16, 32, 256, 0, sizes)[0])
    assert l64 == fp64_rule(driver, 256, sizes)


# A single grid's tile: float64 takes 32x13 (12 waves) when its launch is
# estimated to end at least 2% before that of 16x16, counting a 32x13
# plane-step as 1.45 16x16 ones.  Measured on MI355X (us per 2-step launch,
# 16x16 against 32x13): 176^3 119-120 / 102-106, 200^3 194 / 170-173,
# 256^3 236.7 / 238-240, 320^3 620 / 611, 352^3 787 / 751, 384^3 943 /
# 845, 448^3 1547 / 1504, 512^3 2020 / 1905, 640^3 4759-4936 / 4093-4372,
# 734^3 7547-8884 / 7518-7525; with equal-split chunks (the rule's picks
# here) 320^3 626 (16x16, 64 planes) against 545-555 (32x13, 80), 734^3
# 7750-7812 (16x16, 128) against 6470-6493 (32x13, 105).
@pytest.mark.parametrize("n,eb,want", [
    (256, 8, (16, 16, 128)), (224, 8, (16, 16, 45)), (320, 8, (32, 13, 80)), (96, 8, (16, 16, 8)),
    (176, 8, (32, 13, 30)), (200, 8, (32, 13, 50)), (192, 8, (16, 16, 64)), (734, 8, (32, 13, 105)),
    (352, 8, (32, 13, 118)), (384, 8, (32, 13, 96)), (448, 8, (32, 13, 112)), (416, 8, (16, 16, 70)),
    (512, 8, (32, 13, 128)), (640, 8, (32, 13, 128)), (1024, 8, (32, 13, 128)),
    (256, 4, (16, 32, 64)), (512, 4, (16, 32, 128)), (96, 4, (16, 16, 8)),
])
def test_single_grid_tiles(driver, n, eb, want):
    assert driver.plan(n, eb, 256) == want


def fp64_rule(driver, cus, sizes):
    c16 = driver(16, 16, cus, 0, sizes)[0]
    cw = driver(32, 13, cus, 0, sizes)[0]
    t16, tw = simulate(16, 16, cus, c16, sizes), simulate(32, 13, cus, cw, sizes)
    return (32, 13, cw) if 1.45 * tw < 0.98 * t16 else (16, 16, c16)


@pytest.mark.parametrize("cus", [256, 80])
def test_single_grid_tile_rule(driver, cus):
    for n in range(96, 1025, 32):
        assert driver.plan(n, 8, cus) == fp64_rule(driver, cus, [n]), n


@pytest.mark.parametrize("sizes,want", [
    ([256, 224, 192], (32, 13, 64)),             # three mid-size grids: 32x13
    ([256] * 4, (16, 16, 128)),                  # whole rounds of 16x16 items
    ([64] * 8, (16, 16, 16)),                    # small grids: ragged 32x13 tiles
    ([224, 160, 160, 160, 256, 224, 96, 192, 256, 256, 128, 192, 192, 64, 192, 64],
     (32, 13, 64)),                              # the 16-grid 3-D batch configuration
])
def test_list_tiles(driver, sizes, want):
    _, _, l64, l32 = driver(16, 16, 256, 0, sizes)
    assert l64 == want == fp64_rule(driver, 256, sizes)
    assert l32[:2] == (16, 32)


# The energy reduction's grid: workgroups of 256 columns of a plane of axis
# 0; the closing form holds three per CU, so the planes per workgroup are
# chosen to fill whole rounds of 3 * CUs workgroups (rounds x (planes + 2)).
def energy_cost(dim, n, cus, by):
    cols = n * (n // 2) if dim == 3 else n // 2
    bx = -(-cols // 256)
    c = -(-n // by)
    y = -(-n // c)
    return -(-(bx * y) // (3 * cus)) * (c + 2), bx, y, c


@pytest.mark.parametrize("dim,n,cus", [(3, 256, 256), (3, 512, 256), (3, 96, 256), (3, 34, 256),
                                       (2, 2048, 256), (2, 130, 256), (3, 256, 80), (3, 1024, 256)])
def test_energy_grid_is_the_cheapest_shape(driver, dim, n, cus):
    bx, by, chunk = driver.energy(dim, n, cus)
    assert bx == -(-(n * (n // 2) if dim == 3 else n // 2) // 256)
    assert bx * by <= 2048 and by == -(-n // chunk) and chunk * (by - 1) < n <= chunk * by
    costs = [energy_cost(dim, n, cus, b)[0] for b in range(1, n + 1) if bx * b <= 2048]
    assert energy_cost(dim, n, cus, by)[0] == min(costs)


def test_energy_grid_cases(driver):
    # 256^3 on 256 CUs: 768 workgroups of 43 planes, one round (measured on
    # MI355X, closing form, float64: 167 us against 179 us for 1024
    # workgroups of 32 planes)
    assert driver.energy(3, 256, 256) == (128, 6, 43)
    assert driver.energy(1, 1024, 256) == (0, 0, 0)      # 1-D: no streaming grid
    assert driver.energy(3, 2048, 256) == (0, 0, 0)      # planes beyond 2048 x 256 columns
