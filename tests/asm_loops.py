"""Find loops that contain a workgroup barrier but exit divergently.

Reads AMDGPU assembly written by hipcc -S.  LLVM annotates every basic block
with its innermost loop ("in Loop: Header=BBx_y", "Parent Loop ...", "This
Loop Header").  A loop whose own blocks mask lanes out of the loop
(s_andn2_b64 exec, exec, ...) while it, or a loop nested in it, contains
s_barrier lets some lanes of a wave go round a barrier again while other
lanes wait outside: the workgroup then hangs or reads stale shared data.
"""
import re
import sys
def kernels(path):
    cur=None; lines=[]
    for ln in open(path):
        m=re.match(r'^(_Z\w+):\s*;\s*@', ln)
        if m:
            if cur: yield cur, lines
            cur=m.group(1); lines=[]
        elif cur:
            lines.append(ln.rstrip('\n'))
            if 's_endpgm' in ln:
                yield cur, lines; cur=None; lines=[]
def analyze(lines):
    blocks=[]; cur=None
    for ln in lines:
        m=re.match(r'^(\.LBB\d+_\d+|; %bb\.\d+):', ln)
        if m:
            cur={'name':m.group(1).lstrip('.'), 'loop':None, 'parents':[], 'text':[]}
            blocks.append(cur)
            mm=re.search(r'in Loop: Header=(BB\d+_\d+)', ln)
            if mm: cur['loop']=mm.group(1)
            mm=re.search(r'Parent Loop (BB\d+_\d+)', ln)
            if mm: cur['parents'].append(mm.group(1))
            continue
        if cur is None:
            cur={'name':'entry','loop':None,'parents':[],'text':[]}; blocks.append(cur)
        mm=re.search(r'Parent Loop (BB\d+_\d+)', ln)
        if mm and ln.strip().startswith(';'): cur['parents'].append(mm.group(1))
        if 'This Loop Header' in ln or 'This Inner Loop Header' in ln:
            cur['loop']=cur['name'].replace('LBB','BB')
        cur['text'].append(ln)
    # loop tree
    parent={}
    for b in blocks:
        if b['loop'] and b['loop']==b['name'].replace('LBB','BB'):
            parent[b['loop']]=b['parents'][-1] if b['parents'] else None
    def ancestors(l):
        out=[]
        while l:
            out.append(l); l=parent.get(l)
        return out
    bad=[]
    for L in parent:
        has_bar=False; div=False
        for b in blocks:
            if b['loop'] is None: continue
            anc=ancestors(b['loop'])
            if L in anc:
                if any('s_barrier' in t for t in b['text']): has_bar=True
            if b['loop']==L:
                if any(re.search(r's_andn2_b64 exec, exec', t) for t in b['text']): div=True
        if has_bar and div: bad.append(L)
    return bad

def check_file(path):
    """[(kernel, [loop headers])] of kernels with a divergent loop around a barrier."""
    out = []
    for name, lines in kernels(path):
        bad = analyze(lines)
        if bad:
            out.append((name, bad))
    return out


if __name__ == "__main__":
  rc=0
  for path in sys.argv[1:]:
    for name, bad in check_file(path):
        rc=1; print("DIVERGENT LOOP WITH BARRIER:", name[:90], bad)
  print("checked", sys.argv[1:], "rc", rc)
  sys.exit(rc)
