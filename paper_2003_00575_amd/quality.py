"""Instance-segmentation quality of a labelling against ground-truth instances
(Section IV.B): the Jaccard index of Eq. (5) per instance, its mean, and the
precision P_x of Eq. (6) over the overlap bins 0.50, 0.55, ..., 0.95.

Rules, as the evaluation states them:
  - instances are the ground-truth ids > 0 with at least `min_points` (100)
    measured points; missing pixels (range not > 0 and finite) count for
    neither side;
  - each instance is matched to the cluster (label >= 0) holding most of its
    points, and scored with J = |A n B| / |A u B| over measured points;
  - when one cluster is the best match of several instances
    (under-segmentation), only the instance with the highest J keeps it; the
    others count as not found (J = 0);
  - P_x is the fraction of instances with J >= x; P_mu is the mean of P_x
    over the 10 bins.

    python -m paper_2003_00575_amd.quality [--scans K]

clusters synthetic scenes on the GPU over a grid of thresholds, skip depths
and skip-edge modes (dense, or the Map Connections of Section III.B.2), with
the generator's ground removed and with the ground extraction of Section
III.A, and prints mean IoU and P_mu for each setting.
"""
from __future__ import annotations

import argparse
import json
import sys
from typing import Dict, Iterable, List

import numpy as np

BINS = tuple(round(0.5 + 0.05 * i, 2) for i in range(10))


def instance_ious(labels: np.ndarray, gt: np.ndarray, measured: np.ndarray,
                  min_points: int = 100) -> Dict[int, float]:
    """Jaccard index of every ground-truth instance (id > 0 with at least
    min_points measured points) with its best-overlapping cluster, after the
    under-segmentation rule.  labels, gt: int arrays of one shape; measured:
    bool array of the same shape."""
    lab = np.asarray(labels).ravel()
    g = np.asarray(gt).ravel()
    m = np.asarray(measured, dtype=bool).ravel()
    lab, g = lab[m], g[m]
    ids, counts = np.unique(g[g > 0], return_counts=True)
    inst = [int(i) for i, c in zip(ids, counts) if c >= min_points]
    cl_ids, cl_counts = np.unique(lab[lab >= 0], return_counts=True)
    cl_size = dict(zip(cl_ids.tolist(), cl_counts.tolist()))
    best = {}
    for i in inst:
        sel = g == i
        n_inst = int(sel.sum())
        cand, overlap = np.unique(lab[sel & (lab >= 0)], return_counts=True)
        if cand.size == 0:
            best[i] = (None, 0.0)
            continue
        k = int(np.argmax(overlap))
        c, inter = int(cand[k]), int(overlap[k])
        union = n_inst + cl_size[c] - inter
        best[i] = (c, inter / union)
    # one cluster keeps only its best instance
    owner = {}
    for i, (c, j) in best.items():
        if c is None:
            continue
        if c not in owner or j > best[owner[c]][1]:
            owner[c] = i
    return {i: (j if c is not None and owner.get(c) == i else 0.0) for i, (c, j) in best.items()}


def summarize(ious: Iterable[float]) -> Dict[str, float]:
    """Mean IoU, P_x for every bin (Eq. 6) and their mean P_mu."""
    v = np.asarray(list(ious), dtype=np.float64)
    out = {"instances": int(v.size), "iou_mean": float(v.mean()) if v.size else float("nan")}
    ps = []
    for x in BINS:
        p = float((v >= x).mean()) if v.size else float("nan")
        out[f"P_{x:.2f}"] = p
        ps.append(p)
    out["P_mu"] = float(np.mean(ps)) if v.size else float("nan")
    return out


def literal_first_channel(range_img: np.ndarray, ground: np.ndarray) -> np.ndarray:
    """The ground mask under the literal reading of Section III.A's first-
    channel rule, from the mask of the extended reading: only row 0 takes the
    pair it forms with the row below.  A cell below a missing cell (row > 0)
    then evaluates Eq. (2) with d1 = 0, tan(beta) = -tan(alpha) < 0, which no
    window (its lower end clamped at 0) contains: the cell is kept."""
    r = np.asarray(range_img)
    meas = (r > 0) & np.isfinite(r)
    keep = np.zeros_like(meas)
    keep[..., 1:, :] = ~meas[..., :-1, :]          # the cell above is missing
    return np.asarray(ground, dtype=bool) & ~keep


def _sweep(n_scans: int, thresholds: List[float], depths: List[int], modes=(0,),
           literal_g5: bool = False) -> List[dict]:
    import torch
    from paper_2003_00575_amd import flic, synth
    scans = [synth.large_batch_scan(100 + i, 0.5) for i in range(n_scans)]
    g = synth.ground_tables(scans[0].phi)
    dev = torch.device("cuda:0")
    rng = torch.from_numpy(np.stack([s.range_img for s in scans])).to(dev)
    ours, mask = flic.ground_remove(rng, flic.ground_tables_to_device(g, dev))
    gt_removed = rng.clone()
    gt_removed[torch.from_numpy(np.stack([s.object_id == 0 for s in scans])).to(dev)] = 0.0
    grounds = [("ground truth", gt_removed), ("Section III.A", ours)]
    host_rng = rng.cpu().numpy()
    measured_frac = float(((host_rng > 0) & np.isfinite(host_rng)).mean())
    ext = mask.cpu().numpy().astype(bool)
    gt_ground = np.stack([s.object_id == 0 for s in scans]) & (host_rng > 0) & np.isfinite(host_rng)

    def mask_iou(m: np.ndarray) -> float:
        return float((m & gt_ground).sum() / max(1, (m | gt_ground).sum()))

    print(f"Section III.A removes {ext.mean() / measured_frac:.4f} of the measurements "
          f"(ground truth: {gt_ground.mean() / measured_frac:.4f}); IoU with the true ground "
          f"{mask_iou(ext):.4f}", flush=True)
    if literal_g5:
        lit = literal_first_channel(host_rng, ext)
        print(f"... with the literal first-channel rule: {lit.mean() / measured_frac:.4f}; IoU with the "
              f"true ground {mask_iou(lit):.4f}; cells the readings differ on: "
              f"{(lit != ext).mean() / measured_frac:.4f} of the measurements", flush=True)
        lit_img = rng.clone()
        lit_img[torch.from_numpy(lit).to(dev)] = 0.0
        grounds.append(("III.A literal g5", lit_img))
    ctx = flic.Context(0)
    rows = []
    for ground, imgs in grounds:
        for N, mc in [(N, mc) for N in depths for mc in modes if not (mc and N == 1)]:
            tabs = [synth.make_tables(s.phi, s.W, N) for s in scans]
            cv = [torch.from_numpy(t[0]).to(dev) for t in tabs]
            ch = [torch.from_numpy(t[1]).to(dev) for t in tabs]
            for T in thresholds:
                devs = [flic.DeviceScan(imgs[i], cv[i], ch[i], T, N, None, 0, mc) for i in range(n_scans)]
                ctx.cluster_batched(devs)
                torch.cuda.synchronize()
                ious = []
                for i, s in enumerate(scans):
                    lab = devs[i].labels.cpu().numpy()
                    measured = s.range_img > 0
                    ious.extend(instance_ious(lab, s.object_id, measured).values())
                row = {"ground": ground, "N": N, "maps": mc, "T": T, **summarize(ious)}
                rows.append(row)
                print(f"ground {ground:14s} N={N} {'maps ' if mc else 'dense'} T={T:.2f}: {row['instances']} instances, "
                      f"IoU {row['iou_mean']:.3f}, P_mu {row['P_mu']:.3f}, P_0.50 {row['P_0.50']:.3f}, "
                      f"P_0.75 {row['P_0.75']:.3f}, P_0.95 {row['P_0.95']:.3f}", flush=True)
    return rows


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--scans", type=int, default=16)
    ap.add_argument("--thresholds", default="0.3,0.5,0.8,1.0")
    ap.add_argument("--depths", default="1,2,3,5")
    ap.add_argument("--modes", default="0,1", help="skip-edge modes: 0 dense, 1 Map Connections")
    ap.add_argument("--json", default="")
    ap.add_argument("--literal-g5", action="store_true",
                    help="also score the literal first-channel rule of Section III.A")
    args = ap.parse_args(argv)
    rows = _sweep(args.scans, [float(x) for x in args.thresholds.split(",")],
                  [int(x) for x in args.depths.split(",")], [int(x) for x in args.modes.split(",")],
                  args.literal_g5)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(rows, f)
    return 0


if __name__ == "__main__":
    sys.exit(main())
