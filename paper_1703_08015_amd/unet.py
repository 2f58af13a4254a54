"""3D convolutional U-Net for the learned warm start, assembled from the
liblbm layer kernels (BF16 MFMA convolutions with FP32 accumulation).

Input per voxel: (solid, force direction on fluid voxels) padded to 8
channels.  Output per voxel: 4 values, the steady (rho - rho0, u) divided by
a scale; by the linearity of slow (Stokes) flow in the force, the target is
(rho - rho0, u) * nu / |g| / out_scale.

Levels l = 0..L-1 carry base * 2^l channels.  Encoder level l: two 3x3x3
circular convolutions with ReLU; the second writes into the first half of a
concatenation buffer (the skip).  Between levels: 2x2x2 max pooling.  Bottom
level: two convolutions.  Decoder level l: a 2x2x2 stride-2 transposed
convolution into the second half of the concatenation buffer, then two
convolutions with ReLU.  Head: 1x1x1 convolution to 4 channels (FP32).
Grid edges must be multiples of 2^(L-1).
"""
import math

from . import nn


class Param:
    """FP32 master weights, Adam moments, FP32 gradient and the BF16 copy."""

    def __init__(self, torch, shape, fan_in, device, gen, zero=False, bias=False):
        if zero:
            w = torch.zeros(shape, dtype=torch.float32)
        elif bias:
            w = torch.zeros(shape, dtype=torch.float32)
        else:
            w = torch.randn(shape, generator=gen, dtype=torch.float32) * math.sqrt(2.0 / fan_in)
        self.p = w.to(device)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.g = torch.zeros_like(self.p)
        self.b16 = self.p.to(torch.bfloat16) if not bias else None


class UNet:
    def __init__(self, levels=4, base=24, in_ch=8, out_ch=4, seed=0, device="cuda", out_scale=1.0):
        import torch
        self.torch = torch
        self.L = levels
        self.C = [base * 2 ** l for l in range(levels)]
        self.in_ch, self.out_ch = in_ch, out_ch
        self.out_pad = (out_ch + 7) // 8 * 8  # head gradient rows: BF16, a multiple of 8 wide
        self.device = torch.device(device)
        self.out_scale = out_scale
        # weight gradients run on a second stream beside the backward-data
        # passes (same kernels and results; False keeps one stream), on grids
        # of at least overlap_min_voxels: 96^3 to 128^3 gain 5-9% per training
        # step; at 64^3 two streams took 1.33-1.53 ms from run to run against
        # 1.40 ms on one
        self.overlap = True
        self.overlap_min_voxels = 1 << 19
        self._side = None
        gen = torch.Generator().manual_seed(seed)
        P = lambda shape, fan, **kw: Param(torch, shape, fan, self.device, gen, **kw)
        self.enc = []
        cin = in_ch
        for l in range(levels):
            c = self.C[l]
            self.enc.append([(P((c, 27, cin), 27 * cin), P((c,), 1, bias=True)),
                             (P((c, 27, c), 27 * c), P((c,), 1, bias=True))])
            cin = c
        self.up, self.dec = [], []
        for l in range(levels - 2, -1, -1):
            c, cd = self.C[l], self.C[l + 1]
            self.up.append((P((c, 8, cd), cd), P((c,), 1, bias=True)))
            self.dec.append([(P((c, 27, 2 * c), 27 * 2 * c), P((c,), 1, bias=True)),
                             (P((c, 27, c), 27 * c), P((c,), 1, bias=True))])
        hw = P((self.out_pad, 1, self.C[0]), self.C[0])
        hw.p[out_ch:] = 0.0  # unused rows
        hw.b16 = hw.p.to(torch.bfloat16)
        self.head = (hw, P((self.out_pad,), 1, bias=True))
        self.params = [p for lvl in self.enc for pair in lvl for p in pair]
        self.params += [p for pair in self.up for p in pair]
        self.params += [p for lvl in self.dec for pair in lvl for p in pair]
        self.params += list(self.head)
        self._flatten()
        self.step_count = 0
        self._cache = None

    def _flatten(self):
        """Every parameter's master weights, moments, gradient and BF16 copy
        become views into five flat buffers (segments padded to 8 elements, so
        every BF16 view stays 16-byte aligned): one Adam launch and one
        gradient clear cover the whole network."""
        t = self.torch
        offs, n = [], 0
        for p in self.params:
            offs.append(n)
            n += (p.p.numel() + 7) // 8 * 8
        flat = {k: t.zeros(n, dtype=t.float32, device=self.device) for k in ("p", "m", "v", "g")}
        for p, o in zip(self.params, offs):
            flat["p"][o:o + p.p.numel()].copy_(p.p.reshape(-1))
        p16 = flat["p"].to(t.bfloat16)
        for p, o in zip(self.params, offs):
            k = p.p.numel()
            shape = p.p.shape
            p.p, p.m, p.v, p.g = (flat[name][o:o + k].view(shape) for name in ("p", "m", "v", "g"))
            if p.b16 is not None:
                p.b16 = p16[o:o + k].view(shape)
        self._flat, self._p16 = flat, p16

    # ---- force-linear head -----------------------------------------------------
    def forward_mixed(self, x, direction):
        """With out_ch = 12: per-axis fields mixed by the force direction into
        FP32 (nz, ny, nx, 4)."""
        y = self.forward(x)
        t = self.torch
        shape = tuple(x.shape[:3])
        if getattr(self, "_mixbuf", None) is None or self._mixbuf.shape[:3] != shape:
            self._mixbuf = t.empty(shape + (4,), dtype=t.float32, device=self.device)
        nn.mix(y, direction, self._mixbuf)
        return self._mixbuf

    def backward_mixed(self, dp, ldp, direction):
        t = self.torch
        shape = tuple(dp.shape[:3])
        dy = t.empty(shape + (self.out_pad,), dtype=t.bfloat16, device=self.device)
        nn.mix_backward(dp, ldp, direction, dy, self.out_pad)
        self.backward(dy)

    def n_params(self):
        return int(sum(p.p.numel() for p in self.params) - (self.out_pad - self.out_ch) * (self.C[0] + 1))

    # ---- activations -------------------------------------------------------
    def _alloc(self, shape):
        t = self.torch
        nz, ny, nx = shape
        L = self.L
        if nx % 2 ** (L - 1) or ny % 2 ** (L - 1) or nz % 2 ** (L - 1):
            raise ValueError("grid %s not divisible by %d" % (shape, 2 ** (L - 1)))
        A = {}
        grids = [(nz >> l, ny >> l, nx >> l) for l in range(L)]
        bf = dict(dtype=t.bfloat16, device=self.device)
        for l in range(L):
            g = grids[l]
            c = self.C[l]
            A["e1", l] = t.empty(g + (c,), **bf)
            width = 2 * c if l < L - 1 else c  # concat buffer [skip | up] except at the bottom
            A["cat", l] = t.empty(g + (width,), **bf)
            if l < L - 1:
                A["d1", l] = t.empty(g + (c,), **bf)
                A["d2", l] = t.empty(g + (c,), **bf)
            if l > 0:
                A["pool", l] = t.empty(g + (self.C[l - 1],), **bf)
                A["arg", l] = t.empty(g + (self.C[l - 1],), dtype=t.uint8, device=self.device)
        A["out"] = t.empty(grids[0] + (self.out_ch,), dtype=t.float32, device=self.device)
        return A, grids

    @staticmethod
    def _rows(g):
        return (g[2], g[1], g[0])  # (nx, ny, nz)

    # ---- forward -------------------------------------------------------------
    def forward(self, x):
        """x: BF16 (nz, ny, nx, in_ch).  Returns FP32 (nz, ny, nx, 4)."""
        shape = tuple(x.shape[:3])
        if self._cache is None or self._cache[0] != shape:
            self._cache = (shape,) + self._alloc(shape)
        _, A, grids = self._cache
        self._x = x
        L, C = self.L, self.C
        src, srcld, srcc = x, self.in_ch, self.in_ch
        for l in range(L):
            rows = self._rows(grids[l])
            (w1, b1), (w2, b2) = self.enc[l]
            if l > 0:
                nn.maxpool2(rows, C[l - 1], A["cat", l - 1], 2 * C[l - 1], A["pool", l], C[l - 1], A["arg", l])
                src, srcld, srcc = A["pool", l], C[l - 1], C[l - 1]
            self._fwd(nn.CONV3, nn.IDENT, rows, 27, srcc, C[l], src, srcld, w1.b16, A["e1", l], C[l], bias=b1.p,
                       relu=True)
            width = A["cat", l].shape[-1]
            self._fwd(nn.CONV3, nn.IDENT, rows, 27, C[l], C[l], A["e1", l], C[l], w2.b16, A["cat", l], width,
                       bias=b2.p, relu=True)
        below = A["cat", L - 1]
        for k, l in enumerate(range(L - 2, -1, -1)):
            rows_c, rows = self._rows(grids[l + 1]), self._rows(grids[l])
            uw, ub = self.up[k]
            (w1, b1), (w2, b2) = self.dec[k]
            ldb = below.shape[-1]
            self._fwd(nn.IDENT, nn.SCATTER2, rows_c, 8, C[l + 1], C[l], below, ldb, uw.b16, A["cat", l], 2 * C[l],
                       bias=ub.p, y_offset=C[l])
            self._fwd(nn.CONV3, nn.IDENT, rows, 27, 2 * C[l], C[l], A["cat", l], 2 * C[l], w1.b16, A["d1", l], C[l],
                       bias=b1.p, relu=True)
            self._fwd(nn.CONV3, nn.IDENT, rows, 27, C[l], C[l], A["d1", l], C[l], w2.b16, A["d2", l], C[l],
                       bias=b2.p, relu=True)
            below = A["d2", l]
        hw, hb = self.head
        self._fwd(nn.IDENT, nn.IDENT, self._rows(grids[0]), 1, C[0], self.out_ch, below, C[0], hw.b16, A["out"],
                   self.out_ch, bias=hb.p, y_fp32=True)
        return A["out"]

    # ---- backward ------------------------------------------------------------
    def _conv_backward(self, rows, cin, cout, x, ldx, w, b, dy, lddy, dx, lddx, need_dx=True, gate_ch=None):
        """dy: the gradient of the layer's pre-activation (its ReLU derivative
        already applied where dy was produced).  dx: the gradient of the
        pre-activation of the layer that produced x, i.e. the backward-data
        pass gated by x > 0 on x's first gate_ch (default: all) channels,
        which are that layer's ReLU outputs."""
        self._wg(nn.CONV3, nn.IDENT, rows, 27, cin, cout, x, ldx, dy, lddy, w.g, b.g)
        if need_dx:
            wt = self._wt(w, nn.CONV3, 27, cin, cout)
            self._fwd(nn.CONV3, nn.IDENT, rows, 27, cout, cin, dy, lddy, wt, dx, lddx, gate=x, ldg=ldx,
                       gate_channels=cin if gate_ch is None else gate_ch)

    def _fwd(self, src, dst, rows, taps, cin, cout, x, ldx, w, y, ldy, y_fp32=False, **kw):
        """nn.forward with the shared workspace where the layer splits K (the
        small grids of the coarse levels)."""
        n = nn.forward_workspace(src, dst, rows, taps, cin, cout, ldx, ldy, y_fp32)
        nn.forward(src, dst, rows, taps, cin, cout, x, ldx, w, y, ldy, y_fp32=y_fp32, ws=self._shared_ws(n), **kw)

    def _shared_ws(self, n):
        """A view of n floats of the workspace shared by every layer (grown to
        the largest); None for n = 0."""
        if n == 0:
            return None
        ws = getattr(self, "_ws", None)
        if ws is None or ws.numel() < n:
            ws = self._ws = self.torch.empty(n, dtype=self.torch.float32, device=self.device)
        return ws[:n]

    def _wg(self, src, dst, rows, taps, cin, cout, x, ldx, dy, lddy, dw, db, dy_offset=0):
        """A weight gradient with the workspace it needs (per-block partial
        sums, added in a fixed order).  With overlap, it runs on the side
        stream once everything queued so far on the current stream (dy among
        it) is done, with a workspace of its own, so it overlaps the
        backward-data passes that follow; backward joins the streams at its
        end.  Nothing queued after it writes what it reads: activations are
        not written in backward, and the gradient buffers it reads are only
        accumulated into later on other channels."""
        n = nn.wgrad_workspace(src, dst, rows, taps, cin, cout, ldx, lddy)
        if not self._side:
            nn.wgrad(src, dst, rows, taps, cin, cout, x, ldx, dy, lddy, dw, db, dy_offset=dy_offset,
                     ws=self._shared_ws(n))
            return
        t = self.torch
        self._side.wait_stream(t.cuda.current_stream())
        ws = None
        if n:
            ws = getattr(self, "_side_ws", None)
            if ws is None or ws.numel() < n:
                if ws is not None:
                    # the allocator must not hand the old block out while
                    # side-stream work queued so far may still use it
                    ws.record_stream(self._side)
                ws = self._side_ws = t.empty(n, dtype=t.float32, device=self.device)
            ws = ws[:n]
        nn.wgrad(src, dst, rows, taps, cin, cout, x, ldx, dy, lddy, dw, db, dy_offset=dy_offset, ws=ws,
                 stream=self._side)

    def _wt(self, w, mode, taps, cin, cout):
        """The backward-data weights of a layer, as refreshed by _refresh_wt."""
        return self._wt_cache[("wt", id(w))]

    def _wt_layers(self):
        """(weights, mode, taps, cin, cout) of every layer whose backward-data
        pass runs (all but the first convolution)."""
        L, C = self.L, self.C
        out = [(self.head[0], nn.IDENT, 1, C[0], self.out_pad)]
        for l in range(L - 1):
            idx = L - 2 - l
            (w1, _), (w2, _) = self.dec[idx]
            out += [(w2, nn.CONV3, 27, C[l], C[l]),
                    (w1, nn.CONV3, 27, 2 * C[l], C[l]), (self.up[idx][0], nn.SCATTER2, 8, C[l + 1], C[l])]
        for l in range(L):
            (w1, _), (w2, _) = self.enc[l]
            out.append((w2, nn.CONV3, 27, C[l], C[l]))
            if l > 0:
                out.append((w1, nn.CONV3, 27, C[l - 1], C[l]))
        return out

    def _refresh_wt(self):
        """Every layer's backward-data weights from the current BF16 weights,
        in one launch."""
        t = self.torch
        jobs = []
        for w, mode, taps, cin, cout in self._wt_layers():
            key = ("wt", id(w))
            buf = self._wt_cache.get(key)
            if buf is None:
                buf = self._wt_cache[key] = t.empty((cin, taps, cout), dtype=t.bfloat16, device=self.device)
            jobs.append((mode, taps, cin, cout, w.b16, buf))
        nn.backward_weights_batch(jobs)

    def backward(self, dout):
        """dout: BF16 (nz, ny, nx, out_pad) gradient of the loss wrt the head
        output (channels out_ch.. zero).  Accumulates parameter gradients.
        Every backward-data pass writes the gradient of the pre-activation of
        the layer below it (its ReLU derivative fused as a gate by the
        forward activation), so no separate ReLU-backward pass runs."""
        t = self.torch
        _, A, grids = self._cache
        L, C = self.L, self.C
        if not hasattr(self, "_wt_cache"):
            self._wt_cache = {}
        self._refresh_wt()
        G = self._grads(A, grids)
        use = self.overlap and grids[0][0] * grids[0][1] * grids[0][2] >= self.overlap_min_voxels
        if use and getattr(self, "_side_stream", None) is None:
            self._side_stream = t.cuda.Stream(device=self.device)  # default priority
        self._side = self._side_stream if use else None
        try:
            hw, hb = self.head
            rows0 = self._rows(grids[0])
            below = A["d2", 0] if L > 1 else A["cat", 0]
            ldbelow = C[0] if L > 1 else A["cat", 0].shape[-1]
            self._wg(nn.IDENT, nn.IDENT, rows0, 1, C[0], self.out_pad, below, ldbelow, dout, self.out_pad, hw.g, hb.g)
            wt = self._wt(hw, nn.IDENT, 1, C[0], self.out_pad)
            d_below = G["d2", 0] if L > 1 else G["cat", 0]
            self._fwd(nn.IDENT, nn.IDENT, rows0, 1, self.out_pad, C[0], dout, self.out_pad, wt, d_below, ldbelow,
                       gate=below, ldg=ldbelow, gate_channels=C[0])
            # decoder, top level first (reverse of the forward order)
            for k, l in enumerate(range(0, L - 1)):
                idx = L - 2 - l  # position of level l in self.up / self.dec
                rows, rows_c = self._rows(grids[l]), self._rows(grids[l + 1])
                uw, ub = self.up[idx]
                (w1, b1), (w2, b2) = self.dec[idx]
                self._conv_backward(rows, C[l], C[l], A["d1", l], C[l], w2, b2, G["d2", l], C[l], G["d1", l], C[l])
                # the concat input: only its skip half [0, C) is a ReLU output
                self._conv_backward(rows, 2 * C[l], C[l], A["cat", l], 2 * C[l], w1, b1, G["d1", l], C[l], G["cat", l],
                                    2 * C[l], gate_ch=C[l])
                # transposed conv: input = level l+1 output (d2 of l+1, or the bottom cat buffer)
                if l + 1 == L - 1:
                    xin, ldxin, dxin = A["cat", L - 1], A["cat", L - 1].shape[-1], G["cat", L - 1]
                else:
                    xin, ldxin, dxin = A["d2", l + 1], C[l + 1], G["d2", l + 1]
                self._wg(nn.IDENT, nn.SCATTER2, rows_c, 8, C[l + 1], C[l], xin, ldxin, G["cat", l], 2 * C[l],
                         uw.g, ub.g, dy_offset=C[l])
                wt = self._wt(uw, nn.SCATTER2, 8, C[l + 1], C[l])
                self._fwd(nn.GATHER2, nn.IDENT, rows_c, 8, C[l], C[l + 1], G["cat", l], 2 * C[l], wt, dxin, ldxin,
                           x_offset=C[l], gate=xin, ldg=ldxin, gate_channels=C[l + 1])
            # encoder, bottom level first
            for l in range(L - 1, -1, -1):
                rows = self._rows(grids[l])
                (w1, b1), (w2, b2) = self.enc[l]
                width = A["cat", l].shape[-1]
                self._conv_backward(rows, C[l], C[l], A["e1", l], C[l], w2, b2, G["cat", l], width, G["e1", l], C[l])
                if l > 0:
                    # the pooled gradient is gated by the pooled value, which is the
                    # winning corner's ReLU output, before it joins the skip
                    # gradient already in the first half of cat[l-1]
                    self._conv_backward(rows, C[l - 1], C[l], A["pool", l], C[l - 1], w1, b1, G["e1", l], C[l],
                                        G["pool", l], C[l - 1])
                    nn.maxpool2_backward(rows, C[l - 1], G["pool", l], C[l - 1], A["arg", l], G["cat", l - 1],
                                         2 * C[l - 1], accumulate=True)
                else:
                    self._conv_backward(rows, self.in_ch, C[0], self._x, self.in_ch, w1, b1, G["e1", 0], C[0], None, 0,
                                        need_dx=False)
        finally:
            # join the streams also when a pass raises, so that nothing
            # queued later on the current stream overlaps a weight gradient
            if self._side is not None:
                t.cuda.current_stream().wait_stream(self._side)

    def _grads(self, A, grids):
        t = self.torch
        if getattr(self, "_gcache", None) is None or self._gcache[0] != self._cache[0]:
            G = {}
            for k, v in A.items():
                if isinstance(k, tuple) and k[0] in ("e1", "cat", "d1", "d2", "pool"):
                    G[k] = t.empty_like(v)
            self._gcache = (self._cache[0], G)
        return self._gcache[1]

    def zero_grad(self):
        self._flat["g"].zero_()

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam update of every parameter (a single launch over the flat
        buffers; the BF16 copies, biases' included, are refreshed with it)."""
        self.step_count += 1
        f = self._flat
        nn.adam(f["p"], f["m"], f["v"], f["g"], self._p16, lr, self.step_count, beta1, beta2, eps)

    # ---- state -------------------------------------------------------------------
    def state_dict(self):
        return {"levels": self.L, "base": self.C[0], "out_scale": self.out_scale,
                "params": [p.p.cpu() for p in self.params]}

    def load_state_dict(self, sd):
        for p, v in zip(self.params, sd["params"]):
            p.p.copy_(v.to(self.device))
            if p.b16 is not None:
                p.b16.copy_(p.p.to(self.torch.bfloat16))
        self.out_scale = sd["out_scale"]
