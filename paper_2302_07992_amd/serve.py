"""Serving loop: continuous batching of mixed EMR requests on one GPU.

Two request kinds follow the roles of the reserve-room-before-encryption
framework (Sec. I and III-A):

  EMBED    the content owner encrypts a fresh image with K1 and the data
           hider embeds a payload with K2 (encrypt, then embed);
  RECOVER  the receiver extracts the payload with K2 and restores the image
           with K1 from a marked image (extract, then recover).

Requests arrive over time.  Whenever a launch slot is free the loop admits
the queued requests, oldest first, whose device memory (their outputs plus
the batch's workspace) fits in a fixed pool, and issues them as one batch:
one ``rdhei_run_roles`` call for all of the batch's ops (one table upload),
on the next of a few streams, with the workspace carved from the same pool.  Batches whose completion event has
fired are retired and their memory returned.  Requests that arrive while
other batches run are admitted as soon as a slot and pool memory are free,
so their work overlaps on the device.  Latency is arrival to the completion
event of the request's batch, on the device clock.

Inputs (images, payloads, metadata of marked images) stay resident in device
memory; the keys travel in the job tables.  Torch supplies device memory,
streams and events only: every step of the method runs in librdhei.
"""
from __future__ import annotations

import ctypes
import gc
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import rdhei as R
from .inputs import key_pair, make_image, make_payload, serving_sides

EMBED_REQ, RECOVER_REQ = 0, 1
_ALIGN = 256


def _al(n):
    return (np.asarray(n, dtype=np.int64) + (_ALIGN - 1)) // _ALIGN * _ALIGN


def msg_bytes(nbits):
    """Message buffer bytes the library needs for nbits (vectorised)."""
    nbits = np.asarray(nbits, dtype=np.int64)
    return np.maximum(16, (nbits + 127) // 128 * 16)


@dataclass
class Workload:
    """Requests with resident device inputs (struct of arrays)."""
    kind: np.ndarray        # EMBED_REQ / RECOVER_REQ
    side: np.ndarray        # square image side
    seed: np.ndarray
    nbits: np.ndarray       # payload bits (the image's capacity)
    k1: np.ndarray
    k2: np.ndarray
    in_ptr: np.ndarray      # EMBED: original image; RECOVER: marked image
    msg_ptr: np.ndarray     # EMBED: payload to hide (0 for RECOVER)
    meta_ptr: np.ndarray    # RECOVER: metadata of the marked image (0 for EMBED)
    keep: list = field(default_factory=list)          # tensors that back the pointers
    images: List[torch.Tensor] = field(default_factory=list)    # input image of each request
    payloads: List[torch.Tensor] = field(default_factory=list)  # payload bits of each request
    originals: List[Optional[torch.Tensor]] = field(default_factory=list)  # RECOVER: the plain image

    def __len__(self):
        return len(self.kind)

    @property
    def pixels(self) -> np.ndarray:
        return self.side.astype(np.int64) ** 2

    def out_bytes(self) -> np.ndarray:
        """Pool bytes of each request's outputs."""
        px = self.pixels
        emb = _al(px) + _ALIGN                         # marked image + metadata
        rec = _al(msg_bytes(self.nbits)) + _al(px)     # payload + restored image
        return np.where(self.kind == EMBED_REQ, emb, rec)

    def footprint(self) -> np.ndarray:
        """Admission estimate: outputs plus an upper bound of the workspace.
        Tiled images (sides a multiple of 64) need code records, pyramid,
        tile map and statistics, under 0.1 B/px; other shapes keep a code per
        pixel block of every level, under 0.4 B/px; plus aligned headers."""
        per_px = np.where(self.side % 64 == 0, 10, 2)
        return self.out_bytes() + self.pixels // per_px + 4 * _ALIGN


def make_workload(n: int, seed: int = 0, embed_frac: float = 0.6, sides=None, weights=None,
                  nsin: int = 8, sigma: float = 3.0, device="cuda", ctx: Optional[R.Context] = None,
                  keep_originals: bool = False) -> Workload:
    """n requests of the serving mix, inputs drawn on the device.

    Kinds: EMBED with probability embed_frac, else RECOVER.  Sides: the
    serving mix (256..4096 weighted 30/40/15/10/5) unless `sides`/`weights`
    are given.  Request i uses image seed seed*1_000_003 + i, keys
    key_pair(that seed), and a payload of exactly the image's capacity.
    Capacities and the marked inputs of RECOVER requests are prepared with
    the single-image entry points (not timed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kind = np.where(rng.random(n) < embed_frac, EMBED_REQ, RECOVER_REQ).astype(np.int8)
    if sides is None:
        side = serving_sides(rng, n).astype(np.int32)
    else:
        p = None if weights is None else np.asarray(weights, dtype=np.float64) / np.sum(weights)
        side = rng.choice(np.asarray(sides), size=n, p=p).astype(np.int32)
    seeds = (np.int64(seed) * 1_000_003 + np.arange(n, dtype=np.int64))
    ctx = ctx or R.Context()
    wl = Workload(kind=kind, side=side, seed=seeds, nbits=np.zeros(n, np.int64),
                  k1=np.zeros(n, np.uint64), k2=np.zeros(n, np.uint64), in_ptr=np.zeros(n, np.uint64),
                  msg_ptr=np.zeros(n, np.uint64), meta_ptr=np.zeros(n, np.uint64))
    scratch = {}
    for i in range(n):
        s = int(seeds[i])
        k1, k2 = key_pair(s)
        wl.k1[i], wl.k2[i] = k1, k2
        M = int(side[i])
        img = make_image(s, M, M, nsin, sigma, device)
        meta = R.new_meta(device=device)
        if M not in scratch:
            scratch[M] = torch.empty(M, M, dtype=torch.uint8, device=device)
        enc = torch.empty(M, M, dtype=torch.uint8, device=device) if kind[i] == RECOVER_REQ else scratch[M]
        ctx.encrypt(img, enc, k1, meta, nonce=s)
        torch.cuda.synchronize()
        cap = int(R.read_meta(meta).capacity_bits)
        payload = make_payload(s, cap, device)
        wl.nbits[i] = cap
        msg = torch.zeros(R.msg_bytes(cap), dtype=torch.uint8, device=device)
        msg[: payload.numel()] = payload
        wl.payloads.append(payload)
        if kind[i] == EMBED_REQ:
            wl.in_ptr[i] = img.data_ptr()
            wl.msg_ptr[i] = msg.data_ptr()
            wl.keep += [img, msg]
            wl.images.append(img)
            wl.originals.append(None)
        else:
            ctx.embed(enc, meta, msg, cap, k2)
            wl.in_ptr[i] = enc.data_ptr()
            wl.meta_ptr[i] = meta.data_ptr()
            wl.keep += [enc, meta]
            wl.images.append(enc)
            wl.originals.append(img if keep_originals else None)
    torch.cuda.synchronize()
    return wl


def poisson_arrivals(n: int, rate: float, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of n requests at `rate` per second."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    return np.cumsum(rng.exponential(1.0 / rate, n))


class Arena:
    """Ring allocator over one device buffer; blocks are released in any
    order and their space is reused oldest first."""

    def __init__(self, nbytes: int, device="cuda"):
        self.size = int(nbytes) // _ALIGN * _ALIGN
        raw = torch.empty(self.size + _ALIGN, dtype=torch.uint8, device=device)
        skip = (-raw.data_ptr()) % _ALIGN
        self.buf = raw[skip:skip + self.size]
        self.base = self.buf.data_ptr()
        self.head = 0
        self.blocks = deque()          # [start, end, released]

    def available(self) -> int:
        """Largest contiguous span an allocation could get now."""
        if not self.blocks:
            return self.size
        tail = self.blocks[0][0]
        if self.head > tail:
            return max(self.size - self.head, tail)
        if self.head < tail:
            return tail - self.head
        return 0

    def alloc(self, n: int):
        n = int(-(-n // _ALIGN) * _ALIGN)
        if not self.blocks:
            self.head = 0
        if n > self.available():
            return None
        tail = self.blocks[0][0] if self.blocks else self.size
        start = self.head
        if self.blocks and self.head > tail and self.size - self.head < n:
            start = 0
        blk = [start, start + n, False]
        self.blocks.append(blk)
        self.head = start + n
        if self.head == self.size:
            self.head = 0
        return blk

    def release(self, blk) -> None:
        blk[2] = True
        while self.blocks and self.blocks[0][2]:
            self.blocks.popleft()


@dataclass
class _Batch:
    event: torch.cuda.Event
    block: list
    reqs: np.ndarray
    out: Dict[str, np.ndarray]      # request indices and output offsets in the pool


@dataclass
class ServeResult:
    latency_s: np.ndarray      # per request (nan if rejected)
    wall_s: float
    batches: int
    rejected: int
    pixels: int

    def summary(self) -> dict:
        ok = self.latency_s[np.isfinite(self.latency_s)]
        return {
            "requests": int(len(self.latency_s)), "rejected": int(self.rejected), "batches": int(self.batches),
            "mean_batch": round(len(ok) / max(1, self.batches), 2),
            "p50_ms": round(float(np.percentile(ok, 50)) * 1e3, 4) if len(ok) else None,
            "p99_ms": round(float(np.percentile(ok, 99)) * 1e3, 4) if len(ok) else None,
            "max_ms": round(float(ok.max()) * 1e3, 4) if len(ok) else None,
            "req_per_s": round(len(ok) / self.wall_s, 1),
            "mpx_per_s": round(self.pixels / self.wall_s / 1e6, 1),
            "wall_ms": round(self.wall_s * 1e3, 3),
        }


class Server:
    """Continuous-batching server over librdhei.

    pool_bytes    device memory for outputs and workspaces of requests in flight
    streams       launch streams (one library context each; default one: the
                  device runs one batch at a time, with the next one queued
                  behind it, which keeps the latency tail short)
    max_inflight  batches on the device at once (default 2 per stream)
    max_batch     requests per batch
    per_request   issue each request alone through the single-image entry
                  points on one stream (the baseline), instead of batches
    on_complete   called as on_complete(request_index, outputs) when a
                  request's batch retires, before its memory is reused;
                  outputs maps names to device tensors (views of the pool)
    keystream     keystream family of every request (RDHEI_OPT_KEYSTREAM):
                  R.KEYSTREAM_PHILOX or R.KEYSTREAM_CHACHA20
    """

    def __init__(self, pool_bytes: int = 1 << 30, streams: int = 1, max_inflight: Optional[int] = None,
                 max_batch: int = 2048, per_request: bool = False,
                 on_complete: Optional[Callable[[int, Dict[str, torch.Tensor]], None]] = None, device="cuda",
                 keystream: int = R.KEYSTREAM_PHILOX):
        if per_request:
            streams = 1
        self.per_request = per_request
        self.streams = [torch.cuda.Stream(device=device) for _ in range(streams)]
        self.ctxs = [R.Context() for _ in range(streams)]
        for c in self.ctxs:
            c.set_option(R.OPT_KEYSTREAM, keystream)
        self.arena = Arena(pool_bytes, device)
        self.max_inflight = max_inflight or (64 if per_request else 2 * streams)
        self.max_batch = 1 if per_request else max_batch
        self.on_complete = on_complete
        self.lib = R.load_library()
        self._rr = 0
        self._tmpl = {}

    # ---- one batch -------------------------------------------------------
    @staticmethod
    def _templates(wl: Workload) -> dict:
        """Per-request job rows of the four ops with every field that does not
        depend on where a batch's outputs land, and the requests' output sizes:
        built once per workload, so a batch only gathers rows and sets its
        output pointers."""
        n = len(wl)
        px = wl.pixels
        t = {}
        enc = np.zeros(n, R.JOB_DTYPE)
        enc["inp"] = wl.in_ptr
        enc["key"] = wl.k1
        enc["nonce"] = wl.seed
        enc["height"] = wl.side
        enc["width"] = wl.side
        emb = enc.copy()
        emb["inp"] = 0
        emb["msg"] = wl.msg_ptr
        emb["key"] = wl.k2
        emb["nonce"] = 0
        emb["nbits"] = wl.nbits
        ext = np.zeros(n, R.JOB_DTYPE)
        ext["inp"] = wl.in_ptr
        ext["meta"] = wl.meta_ptr
        ext["key"] = wl.k2
        ext["nbits"] = wl.nbits
        ext["height"] = wl.side
        ext["width"] = wl.side
        rec = ext.copy()
        rec["nbits"] = 0
        rec["key"] = wl.k1
        t.update(enc=enc, emb=emb, ext=ext, rec=rec)
        # outputs back to back: EMBED (image, meta), then RECOVER (msg, image)
        t["img_al"] = _al(px)
        t["sz_e"] = t["img_al"] + _ALIGN
        t["sz_r_msg"] = _al(msg_bytes(wl.nbits))
        t["sz_r"] = t["sz_r_msg"] + t["img_al"]
        t["is_e"] = wl.kind == EMBED_REQ
        return t

    def _tables(self, wl: Workload, idx: np.ndarray, base: int):
        """Job tables of the four ops and the output offsets of a batch whose
        outputs start at device address `base` (256-byte aligned)."""
        t = self._tmpl.get(id(wl))
        if t is None or t["wl"] is not wl:
            t = self._templates(wl)
            t["wl"] = wl
            self._tmpl = {id(wl): t}
        me = t["is_e"][idx]
        e = idx[me]
        r = idx[~me]
        sz_e = t["sz_e"][e]
        sz_r = t["sz_r"][r]
        cs_e = np.cumsum(sz_e)
        end_e = int(cs_e[-1]) if len(e) else 0
        off_e = cs_e - sz_e
        off_r = end_e + np.cumsum(sz_r) - sz_r
        total = end_e + (int(sz_r.sum()) if len(r) else 0)
        out = {"e": e, "r": r, "img_e": off_e, "meta_e": off_e + t["img_al"][e], "msg_r": off_r,
               "img_r": off_r + t["sz_r_msg"][r]}
        tabs = []
        if len(e):
            enc = t["enc"][e]
            enc["out"] = base + out["img_e"]
            enc["meta"] = base + out["meta_e"]
            emb = t["emb"][e]
            emb["out"] = enc["out"]
            emb["meta"] = enc["meta"]
            tabs += [(R.OP_ENCRYPT, enc, ("out", "meta")), (R.OP_EMBED, emb, ("out", "meta"))]
        if len(r):
            ext = t["ext"][r]
            ext["msg"] = base + out["msg_r"]
            rec = t["rec"][r]
            rec["out"] = base + out["img_r"]
            tabs += [(R.OP_EXTRACT, ext, ("msg",)), (R.OP_RECOVER, rec, ("out",))]
        return tabs, out, total

    def _issue_single(self, ctx, sp, op, j) -> None:
        """One request, one op, through the single-image entry points."""
        lib, h = self.lib, ctx.h
        M = int(j["height"])
        if op == R.OP_ENCRYPT:
            rc = lib.rdhei_encrypt(h, int(j["inp"]), int(j["out"]), M, M, int(j["key"]), int(j["nonce"]), R.EMR,
                                   int(j["meta"]), sp)
        elif op == R.OP_EMBED:
            rc = lib.rdhei_embed(h, int(j["out"]), M, M, R.EMR, int(j["meta"]), int(j["msg"]), int(j["nbits"]),
                                 int(j["key"]), sp)
        elif op == R.OP_EXTRACT:
            rc = lib.rdhei_extract(h, int(j["inp"]), M, M, R.EMR, int(j["meta"]), int(j["msg"]), int(j["nbits"]),
                                   int(j["key"]), sp)
        else:
            rc = lib.rdhei_recover(h, int(j["inp"]), M, M, R.EMR, int(j["meta"]), int(j["out"]), int(j["key"]), sp)
        R._check(rc, "single-image call")

    def _launch(self, wl: Workload, idx: np.ndarray, est: int) -> Optional[_Batch]:
        """Allocate and issue one batch; None if the pool cannot hold it now."""
        si = self._rr
        ctx, st = self.ctxs[si], self.streams[si]
        # table contents depend on the output base only through its alignment,
        # so size the workspace with the pool base, then shift the pointers
        tabs, out, total = self._tables(wl, idx, self.arena.base)
        ws = 0 if self.per_request else int(_al(ctx.roles_workspace_size([(op, t) for op, t, _ in tabs])))
        blk = self.arena.alloc(max(ws + total, est))
        if blk is None:
            return None
        self._rr = (self._rr + 1) % len(self.streams)
        base = self.arena.base + blk[0]
        shift = base + ws - self.arena.base
        sp = ctypes.c_void_p(st.cuda_stream)
        for op, t, fields in tabs:
            for f in fields:
                t[f] += np.uint64(shift)
            if self.per_request:
                self._issue_single(ctx, sp, op, t[0])
        if not self.per_request:
            # every op of the batch in one call: one table upload
            ctx.run_roles([(op, t) for op, t, _ in tabs], base, ws, st)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(st)
        for k in ("img_e", "meta_e", "msg_r", "img_r"):
            out[k] = out[k] + shift
        return _Batch(ev, blk, idx, out)

    def _views(self, wl: Workload, b: _Batch):
        buf = self.arena.buf
        for j, i in enumerate(b.out["e"]):
            M = int(wl.side[i])
            o, m = int(b.out["img_e"][j]), int(b.out["meta_e"][j])
            yield int(i), {"marked": buf[o:o + M * M].view(M, M), "meta": buf[m:m + R.META_BYTES]}
        for j, i in enumerate(b.out["r"]):
            M = int(wl.side[i])
            o, m = int(b.out["img_r"][j]), int(b.out["msg_r"][j])
            yield int(i), {"recovered": buf[o:o + M * M].view(M, M),
                           "payload": buf[m:m + int(msg_bytes(wl.nbits[i]))]}

    # ---- the loop --------------------------------------------------------
    def run(self, wl: Workload, arrivals: np.ndarray, count: Optional[int] = None) -> ServeResult:
        """Serve the first `count` (default all) of wl's requests, arriving at
        `arrivals` (seconds, ascending).  The interpreter's cyclic garbage
        collector is paused meanwhile (the loop makes small objects per batch;
        a collection in the middle of a run stalls every request queued)."""
        was = gc.isenabled()
        gc.disable()
        try:
            return self._run(wl, arrivals, count)
        finally:
            if was:
                gc.enable()

    def _run(self, wl: Workload, arrivals: np.ndarray, count: Optional[int] = None) -> ServeResult:
        n = len(wl) if count is None else int(count)
        arrivals = np.asarray(arrivals, dtype=np.float64)
        assert len(arrivals) == n and np.all(np.diff(arrivals) >= 0)
        est = wl.footprint()
        lat = np.full(n, np.nan)
        inflight: List[_Batch] = []
        done = rejected = batches = 0
        qh = nxt = 0
        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.streams[0])
        t0 = time.perf_counter()
        finished = []
        while done + rejected < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                nxt += 1
            # retire finished batches
            k = 0
            while k < len(inflight):
                b = inflight[k]
                if b.event.query():
                    inflight.pop(k)
                    finished.append(b)
                    if self.on_complete is not None:
                        for i, views in self._views(wl, b):
                            self.on_complete(i, views)
                    self.arena.release(b.block)
                    done += len(b.reqs)
                else:
                    k += 1
            # admit oldest first while pool memory and a launch slot are free
            while qh < nxt and len(inflight) < self.max_inflight:
                if est[qh] > self.arena.size:
                    rejected += 1          # can never fit the pool
                    qh += 1
                    continue
                avail = self.arena.available()
                hi = min(nxt, qh + self.max_batch)
                cum = np.cumsum(est[qh:hi])
                take = int(np.searchsorted(cum, avail, side="right"))
                if take == 0:
                    break
                b = self._launch(wl, np.arange(qh, qh + take), int(cum[take - 1]))
                while b is None and not inflight and take > 1:
                    take //= 2        # the exact workspace outgrew the estimate
                    b = self._launch(wl, np.arange(qh, qh + take), int(cum[take - 1]))
                if b is None:
                    if not inflight:
                        rejected += 1      # larger than the whole pool
                        qh += 1
                        continue
                    break
                inflight.append(b)
                batches += 1
                qh += take
        torch.cuda.synchronize()
        wall_dev = 0.0
        for b in finished:
            t = ref.elapsed_time(b.event) / 1e3
            lat[b.reqs] = t - arrivals[b.reqs]
            wall_dev = max(wall_dev, t)
        wall = max(wall_dev, 1e-9)
        px = int(wl.pixels[:n][np.isfinite(lat)].sum())
        return ServeResult(lat, wall, batches, rejected, px)
