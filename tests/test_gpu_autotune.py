"""The tile-shape x batch autotuner's search, with a stand-in workload whose
time is set per candidate (a device spin of a chosen length): the search must
return the candidate with the shortest spin and skip the invalid tilings."""
import pytest
import torch

from paper_2606_30436_amd.autotune import autotune

TILES = [(16, 16), (32, 16), (16, 32)]
BATCHES = [32, 64, 128]


@pytest.mark.gpu
def test_autotune_picks_the_fastest():
    cost = {}
    for i, t in enumerate(TILES):
        for j, b in enumerate(BATCHES):
            cost[(t, b)] = 400_000 + 150_000 * ((3 * i + 5 * j) % 7)
    fastest = min((k for k in cost if not (k[0][0] * k[0][1] == 512 and k[1] > 64)), key=cost.get)
    cost[fastest] = 200_000
    cur = {}

    def set_tiling(tile, batch):
        cur["k"] = (tuple(tile), int(batch))

    def run():
        torch.cuda._sleep(cost[cur["k"]])

    best, table = autotune(run, set_tiling, TILES, BATCHES, reps=3, cache_path=None)
    assert best == fastest
    assert "32x16/128" not in table and "16x32/128" not in table and "16x16/128" in table
    assert len(table) == len(TILES) * len(BATCHES) - 2
    assert table[f"{fastest[0][0]}x{fastest[0][1]}/{fastest[1]}"] == min(table.values())
